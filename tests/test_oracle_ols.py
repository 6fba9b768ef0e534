"""Pins for oracle.ols (Definition 2.1, Theorem 2.2): the QR oracle is checked
against exact rational arithmetic, closed forms, exact AR recursions and
independent factorisations, so that a dropped term, a wrong index or a
transposed operand in it fails one of these."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def _exact_normal_solution(y, p):
    """Solve X^T X phi = X^T b in exact rationals (Gaussian elimination);
    None if X^T X is singular.  X and b are written out here from eq. (xphi)
    independently of oracle.lag_matrix."""
    n = len(y)
    rows = [[Fraction(y[t - 1 - j]) for j in range(p)] for t in range(p, n)]
    rhs = [Fraction(y[t]) for t in range(p, n)]
    G = [[sum(r[a] * r[c] for r in rows) for c in range(p)] for a in range(p)]
    h = [sum(r[a] * bb for r, bb in zip(rows, rhs)) for a in range(p)]
    A = [G[a] + [h[a]] for a in range(p)]
    for col in range(p):
        piv = next((r for r in range(col, p) if A[r][col] != 0), None)
        if piv is None:
            return None
        A[col], A[piv] = A[piv], A[col]
        for r in range(p):
            if r != col and A[r][col] != 0:
                f = A[r][col] / A[col][col]
                A[r] = [a - f * c for a, c in zip(A[r], A[col])]
    return [A[i][p] / A[i][i] for i in range(p)]


@pytest.mark.parametrize("p", [1, 2, 3])
def test_bruteforce_enumeration_exact_rational(p):
    """Every integer series in {-1,0,1}^n (n = 2p+1 .. 7): the FP64 QR oracle
    matches the exact rational normal-equation solution to 1e-12 relative
    (rank-deficient cases skipped; Theorem 2.2)."""
    checked = 0
    for n in range(2 * p + 1, 8):
        for y in itertools.product((-1, 0, 1), repeat=n):
            exact = _exact_normal_solution(y, p)
            if exact is None:
                continue
            X, _ = oracle.lag_matrix(np.array(y, float), p)
            if np.linalg.matrix_rank(X) < p:
                continue
            got = oracle.fit_qr(np.array(y, float), p)["phi"]
            ex = np.array([float(e) for e in exact])
            k = oracle.kappa(oracle.qr_r(X))
            scale = max(np.linalg.norm(ex), 1.0)
            assert np.linalg.norm(got - ex) <= 1e-14 * max(k, 1.0) ** 2 * scale * 10, (y, p)
            checked += 1
    assert checked > 50


def test_p1_closed_form(rng):
    """p = 1: phi = sum_t y_t y_{t+1} / sum_t y_t^2 over t = 1..n-1 (the same
    denominator as the exact p = 1 leverage of Section 3.1)."""
    y = rng.standard_normal(500)
    phi = oracle.fit_qr(y, 1)["phi"][0]
    closed = np.dot(y[:-1], y[1:]) / np.dot(y[:-1], y[:-1])
    assert abs(phi - closed) <= 1e-14 * abs(closed) * 10


@pytest.mark.parametrize("K,const", [(1, False), (2, False), (2, True), (4, True), (6, False)])
def test_noise_free_recovery(K, const):
    """A sum of K cosines (+ a constant) obeys an AR(2K [+1]) recursion with
    zero innovations, so the OLS fit recovers its coefficients exactly and
    leaves zero residual."""
    freqs = np.linspace(0.35, 2.6, K)
    amps = np.linspace(1.0, 2.0, K)
    phases = np.linspace(0.1, 1.3, K)
    y = synth.sinusoid_series(2000, freqs, amps, phases, 0.7 if const else None)
    p = 2 * K + (1 if const else 0)
    truth = synth.sinusoid_coefficients(freqs, const)
    fit = oracle.fit_qr(y, p)
    err = oracle.rel_error(fit["phi"], truth)
    assert err <= 1e-16 * fit["kappa"] * 100 + 1e-13, (err, fit["kappa"])
    assert fit["rnorm"] <= 1e-10 * np.linalg.norm(y)


def test_normal_equation_orthogonality(rng):
    """Theorem 2.2: X^T r = 0 at the OLS solution."""
    for p in (2, 5, 11):
        y = synth.ar_series(3000, p, rng, 0.3, 0.8)
        fit = oracle.fit_qr(y, p)
        assert fit["kappa"] < 1e4
        assert oracle.normal_residual(y, p, fit["phi"]) <= 1e-13


def test_residual_norm_matches_last_diagonal(rng):
    y = synth.ar_series(1500, 6, rng, 0.3, 0.9)
    fit = oracle.fit_qr(y, 6)
    assert abs(fit["rnorm"] - oracle.residual_norm(y, 6, fit["phi"])) <= 1e-12 * fit["rnorm"]


def test_lapack_vs_householder_vs_svd(rng):
    """Three independent factorisations agree on well-conditioned inputs."""
    for p in (1, 3, 8):
        y = synth.ar_series(400, p, rng, 0.2, 0.7)
        X, b = oracle.lag_matrix(y, p)
        Q, R = oracle.householder_qr(np.column_stack([X, b]))
        assert np.allclose(Q @ R, np.column_stack([X, b]), atol=1e-12 * np.abs(y).max())
        assert np.allclose(Q.T @ Q, np.eye(p + 1), atol=1e-13)
        phi_h = np.linalg.solve(R[:p, :p], R[:p, p])
        phi_q = oracle.fit_qr(y, p)["phi"]
        phi_s = oracle.fit_svd(X, b)
        assert oracle.rel_error(phi_q, phi_s) < 1e-12
        assert oracle.rel_error(phi_h, phi_s) < 1e-12
        # LAPACK R equals the hand-written R up to row signs
        RL = oracle.qr_r(np.column_stack([X, b]))
        sgn = np.sign(np.diag(RL)) * np.sign(np.diag(R))
        assert np.allclose(RL, sgn[:, None] * R, atol=1e-11 * np.abs(R).max())


def test_rank_deficient_min_norm():
    """Theorem 2.2 singular case: a constant series with p = 2 gives rank-1 X;
    the SVD route returns the minimum-norm solution, equal to pinv(X) b."""
    y = np.full(50, 3.0)
    X, b = oracle.lag_matrix(y, 2)
    assert np.linalg.matrix_rank(X) == 1
    x = oracle.fit_svd(X, b)
    assert np.allclose(x, [0.5, 0.5])
    assert np.allclose(X @ x, b)


def test_rel_error_is_phierr_without_100():
    assert oracle.rel_error([1.0, 1.0], [1.0, 0.0]) == pytest.approx(1.0)
    assert oracle.rel_error([3.0, 4.0], [3.0, 4.0]) == 0.0


def test_tri_inverse(rng):
    R = np.triu(rng.standard_normal((7, 7))) + 5 * np.eye(7)
    assert np.allclose(oracle.tri_inverse(R) @ R, np.eye(7), atol=1e-13)
