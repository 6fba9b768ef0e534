"""Row sampling, sketch rows and the randomized Hadamard map (oracle; test
infrastructure only).  Random numbers are inputs: every function takes its
uniform draws in [0, 1) as an array, so the GPU path and the oracle can be fed
the same draws.

uniform_rows: Algorithm 1's i.i.d. uniform trials; row i = floor(u m), and the
  sampled row is rescaled by sqrt(m / c).
leverage_sample: Algorithm 2 / eq. (ldist): pi_i = l_i / sum_k l_k, c draws
  with replacement, each sampled row rescaled by 1 / sqrt(c pi_i) (the
  sampling-and-rescaling rule of Section 2.1.2).  A draw u picks the first row
  whose running score total exceeds u * total (inverse CDF, the running total
  accumulated in row order).
sketch_rows: the sampled, rescaled rows of [X | b] (eq. (OLSc) with S applied).
rh_levels, rh_level_mask: the nested uniform halvings of Algorithm 4 (repeated
  halving): row r belongs to level i when its draw u_r < 2^-i (so each level
  is a uniform half of the one before, in expectation), with as many levels
  as halvings of m rows until a level holds no more than c rows.
rh_sketch: Algorithm 4 end to end.  The smallest level is stood for by c
  uniform row trials (scale sqrt(m/c)); going up, level i's rows are scored
  with the approximate generalised leverage scores of eq. (glev) with respect
  to the sketch of level i + 1 (R from one shifted Cholesky QR sweep of that
  sketch, shifted_r, Omega = R^{-1} Pi^T with one k x p JL map Pi for every
  level), rows outside level i get score zero, and c rows are drawn from the
  scores (leverage_sample with that level's draws) to form level i's sketch;
  level 0 is all rows, and its sketch is the result.
compressed_solution: the compressed (sketch-and-solve) estimator of Section
  2.1, the minimiser of ||S X phi - S b|| (eq. (OLSc)), by Householder QR of
  S X.
hadamard: Definition 2.4, H_0 = 1 and H_m = [[H, H], [H, -H]] / sqrt(2),
  of size 2^m (the paper's size label is garbled; H_m is 2^m x 2^m here).
srht_map: a k x p subsampled randomized Hadamard map sqrt(P/k) S H D on the
  p-vector zero-padded to P = 2^ceil(log2 p) (Algorithm 1's construction with
  random signs D and k uniform row trials S), restricted to its first p columns.
jl_omega: Omega = R^{-1} Pi^T, the k columns whose row products give the
  approximate generalised leverage scores of eq. (glev).

Parity pins (tests/test_oracle_sketch.py): rh_sketch with one level is the
one-level leverage sketch (uniform trials, eq. (glev) scores w.r.t. them,
leverage sampling) built step by step; rows drawn at a level above 0 lie in
that level and level 0 draws from all rows; with k = p and Pi = I its top-level
scores are the exact generalised scores of Definition 3.6 w.r.t. the level
below.  The compressed estimator with every
row at unit scale equals the full least-squares solution, recovers the
coefficients of a noise-free AR series from any sampled rows, has the p = 1
closed form sum s^2 x b / sum s^2 x^2, and ignores a common row scale and row
duplication; a hand-worked inverse-CDF example;
E[S^T S] = I for the rescaled sampling matrix (Monte Carlo); H_m orthonormal
and H_1 written out; E||Pi x||^2 = ||x||^2 for the SRHT map.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .toeplitz import lag_matrix, matvec


def uniform_rows(u, m: int, c: int | None = None):
    """Row indices floor(u m) (clamped to m-1) and the common scale sqrt(m/c)."""
    u = np.asarray(u, np.float64)
    c = u.size if c is None else c
    idx = np.minimum(np.floor(u * m).astype(np.int64), m - 1)
    scale = np.full(idx.size, np.sqrt(m / c))
    return idx, scale


def leverage_sample(scores, u, c: int | None = None):
    """Inverse-CDF draws from pi = scores / sum(scores) and scales 1/sqrt(c pi)."""
    s = np.asarray(scores, np.float64)
    u = np.asarray(u, np.float64)
    c = u.size if c is None else c
    running = np.cumsum(s)
    total = running[-1]
    idx = np.searchsorted(running, u * total, side="right")
    idx = np.minimum(idx, s.size - 1)
    pi = s[idx] / total
    scale = 1.0 / np.sqrt(c * pi)
    return idx.astype(np.int64), scale


def sketch_rows(y, p: int, idx, scale) -> np.ndarray:
    """[S X | S b]: row t is scale_t * [X(idx_t, :), b(idx_t)]; shape (c, p+1)."""
    X, b = lag_matrix(y, p)
    idx = np.asarray(idx, np.int64)
    scale = np.asarray(scale, np.float64)
    return np.column_stack([X[idx, :], b[idx]]) * scale[:, None]


def rh_levels(m: int, c: int) -> int:
    """Halvings of m rows until a level holds no more than c rows (>= 1)."""
    levels = 1
    while (m >> levels) > c:
        levels += 1
    return levels


def rh_level_mask(u, level: int) -> np.ndarray:
    """Rows of level `level`: u_r < 2^-level (u: one uniform draw per row)."""
    return np.asarray(u, np.float64) < 2.0 ** (-level)


def compressed_solution(A) -> np.ndarray:
    """Minimiser of ||S X phi - S b|| for the sketch A = [S X | S b] (c x (p+1),
    sketch_rows): the compressed estimator of Section 2.1, eq. (OLSc)."""
    A = np.asarray(A, np.float64)
    Q, R = sla.qr(A[:, :-1], mode="economic")
    return sla.solve_triangular(R, Q.T @ A[:, -1])


def hadamard(mexp: int) -> np.ndarray:
    """Normalised Hadamard matrix H_mexp of size 2^mexp (Definition 2.4)."""
    H = np.array([[1.0]])
    for _ in range(mexp):
        H = np.block([[H, H], [H, -H]]) / np.sqrt(2.0)
    return H


def srht_map(p: int, k: int, u_signs, u_rows) -> np.ndarray:
    """k x p map sqrt(P/k) S H_P D (first p columns); D_jj = +1 if u_signs[j] < 0.5
    else -1 (j < P); S picks rows floor(u_rows[t] * P)."""
    P = 1
    while P < p:
        P *= 2
    H = hadamard(int(np.log2(P)))
    d = np.where(np.asarray(u_signs, np.float64)[:P] < 0.5, 1.0, -1.0)
    rows = np.minimum(np.floor(np.asarray(u_rows, np.float64)[:k] * P).astype(np.int64), P - 1)
    Pi = np.sqrt(P / k) * H[rows, :] * d[None, :]
    return Pi[:, :p]


def sketch_r(A, p: int) -> np.ndarray:
    """R of a sketch's first p columns with a non-negative diagonal, the
    unique upper-triangular factor with R^T R = A^T A.  A QR fixes R only up
    to the signs of its rows; the generalised scores of eq. (glev) use R only
    through R^{-1}, but once a JL map multiplies R^{-1} the approximate scores
    depend on those signs (R^{-1} D Pi^T is another map for every sign
    matrix D), so they are fixed here."""
    R = sla.qr(np.asarray(A, np.float64)[:, :p], mode="r")[0][:p, :p]
    return R * np.where(np.diag(R) < 0, -1.0, 1.0)[:, None]


def shifted_r(A, p: int) -> np.ndarray:
    """The factor that approximate scores are taken with respect to: R[:p, :p]
    of one sweep of shifted Cholesky QR (Fukaya, Kannan, Nakatsukasa,
    Yamamoto, Yanagisawa, SIAM J. Sci. Comput. 2020) of the q-column sketch A,
    i.e. the transposed Cholesky factor of A^T A + s I with the shift
    s = 11 (c' q + q (q + 1)) u tr(A^T A), u = 2^-53 and c' the sketch's row
    count rounded up to a multiple of 16 (zero rows padding it to the row
    tiles).  It equals the QR factor of A with a non-negative diagonal
    (sketch_r) up to relative O(s / sigma_min(A)^2); the approximate scores
    are defined with respect to this factor, which exists for any A."""
    A = np.asarray(A, np.float64)
    q = A.shape[1]
    crows = -(-A.shape[0] // 16) * 16
    G = A.T @ A
    s = 11.0 * (crows * q + q * (q + 1)) * 2.0 ** -53 * np.trace(G)
    L = np.linalg.cholesky(G + s * np.eye(q))
    return L.T[:p, :p]


def jl_omega(R, Pi) -> np.ndarray:
    """Omega = R^{-1} Pi^T (p x k) for upper-triangular R."""
    return sla.solve_triangular(np.asarray(R, np.float64), np.asarray(Pi, np.float64).T,
                                lower=False)


def rh_sketch(y, p: int, c: int, u_uniform, u_level, Pi, level_draws):
    """Algorithm 4 (module doc).  u_uniform: c uniforms of the smallest
    level's trials; u_level: one uniform per row (the nested halvings);
    Pi: k x p JL map; level_draws[i]: c uniforms of level i's draws, for
    i < rh_levels(m, c).  Returns (A, idx, scale, levels): the final sketch
    [S X | S b], its rows and scales, and the number of levels."""
    y = np.asarray(y, np.float64)
    m = y.size - p
    levels = rh_levels(m, c)
    idx, scale = uniform_rows(u_uniform, m, c)
    A = sketch_rows(y, p, idx, scale)
    for lev in range(levels - 1, -1, -1):
        Omega = jl_omega(shifted_r(A, p), Pi)
        Z = np.column_stack([matvec(y, p, Omega[:, q]) for q in range(Omega.shape[1])])
        s = np.sum(Z * Z, axis=1)
        if lev > 0:
            s = np.where(rh_level_mask(u_level, lev), s, 0.0)
        idx, scale = leverage_sample(s, level_draws[lev], c)
        A = sketch_rows(y, p, idx, scale)
    return A, idx, scale, levels
