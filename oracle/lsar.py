"""LSAR: PACF through approximate leverage-score sampling (oracle; test
infrastructure only).

Section 3.1 (LSAR algorithm), Definition of the approximate leverage scores,
eqs. (FALS), (FAR), (FASD), and Algorithm 3.  The lags h = 1 .. pmax are
visited in order; lag h fits AR(h) on the series prefix of n - pmax + h
samples, so every lag has R = n - pmax rows, and row i of lag h's lag matrix
is (y[h-1+i], ..., y[i]) with response y[h+i] (0-based).  Row i of lag h is
therefore row i of lag h - 1 with lag h - 1's response put in front of it,
which is what makes the recursion of eq. (FALS) a statement about the same
rows at every lag.

Scores of lag h (the rows' approximate leverage scores for the lag matrix X_h):
  h = 1: the exact scores y[i]^2 / sum_{t<R} y[t]^2 (the one-column case of
         Definition 2.6, the closed form given with Definition 3.4);
  h > 1: l_h(i) = l_{h-1}(i) + r_{h-1}(i)^2 / ||r_{h-1}||^2 (eq. (FALS)), with
         r_{h-1} = X_{h-1} phi_{h-1} - b_{h-1} over all R rows (eq. (FAR)) and
         phi_{h-1} the compressed solution of lag h - 1.  (h = 2 is the
         "quasi-approximate" case: l_1 is exact there.)
Every increment sums to one, so the scores of lag h sum to h and eq. (FASD)'s
pi_h = l_h / h is a distribution.

Per lag (Algorithm 3): sample c rows with replacement from pi_h by the inverse
CDF of the running total (leverage_sample, rows rescaled 1/sqrt(c pi)), solve
the compressed problem of eq. (OLSc) on [S X_h | S b_h] (compressed_solution),
and read the PACF estimate tau_h as the last coefficient.  The order estimate
is the largest h with |tau_h| >= 1.96 / sqrt(c).

Random numbers are inputs: draws[h-1] holds lag h's c uniforms in [0, 1).

Readings (garbles of the printed algorithm): "Set h = 0" is read as p = 0
(the loop variable is p); the PACF estimate at lag p is taken after the
compressed fit of that lag (the last coefficient of its solution), since it
needs that fit; the sampling distribution uses the scores of the lag being
fitted, and c is a fixed input (the experiments use c = 2000 at every lag).

Parity pins (tests/test_oracle_lsar.py): with each lag's exact least-squares
solution in place of the compressed one, the recursion reproduces the exact
leverage scores (hat-matrix diagonal, Definition 2.6) of every lag's lag
matrix (the rank-one update of the hat matrix when lag h - 1's response joins
as a column); the lag-1 scores equal Definition 2.6 on the one-column matrix;
the scores of lag h sum to h for any coefficients; with the sampled rows
given, tau equals pacf_compressed on the same rows; the order rule.
"""
from __future__ import annotations

import numpy as np

from .sketch import compressed_solution, leverage_sample, sketch_rows


def lag_rows(y, pmax: int, h: int):
    """Lag h's prefix of the series, y[: n - pmax + h] (R = n - pmax rows)."""
    y = np.asarray(y, np.float64)
    return y[: y.size - pmax + h]


def scores_lag1(y, pmax: int) -> np.ndarray:
    """Exact scores of lag 1: y[i]^2 / sum_{t < R} y[t]^2, i < R."""
    y = np.asarray(y, np.float64)
    R = y.size - pmax
    col = y[:R]
    return col * col / np.dot(col, col)


def residual(y, pmax: int, h: int, phi) -> np.ndarray:
    """eq. (FAR): r_h = X_h phi - b_h over all R rows of lag h, straight from
    the indexing X_h[i, j] = y[h-1+i-j], b_h[i] = y[h+i]."""
    y = np.asarray(y, np.float64)
    R = y.size - pmax
    phi = np.asarray(phi, np.float64)
    i = np.arange(R)
    r = -y[h + i]
    for j in range(h):
        r = r + phi[j] * y[h - 1 + i - j]
    return r


def scores_next(scores_prev, r_prev) -> np.ndarray:
    """eq. (FALS) for h > 1: l_h = l_{h-1} + r_{h-1}^2 / ||r_{h-1}||^2."""
    r = np.asarray(r_prev, np.float64)
    return np.asarray(scores_prev, np.float64) + r * r / np.dot(r, r)


def lsar_pacf(y, pmax: int, c: int, draws, solve=None, keep_scores: bool = False):
    """Algorithm 3 over lags 1..pmax.  Returns a dict with tau (pmax), the
    per-lag coefficient vectors phi[h-1], the sampled rows (idx, scale) of
    every lag, order (the largest h with |tau_h| >= 1.96 / sqrt(c)), and with
    keep_scores every lag's scores.

    `solve(y_prefix, h, idx, scale)` replaces the compressed solve when given
    (the pins use the exact least-squares solution there)."""
    y = np.asarray(y, np.float64)
    tau, phis, rows, kept = np.zeros(pmax), [], [], []
    scores = None
    for h in range(1, pmax + 1):
        if h == 1:
            scores = scores_lag1(y, pmax)
        else:
            scores = scores_next(scores, residual(y, pmax, h - 1, phis[-1]))
        if keep_scores:
            kept.append(scores)
        idx, scale = leverage_sample(scores, draws[h - 1], c)
        yy = lag_rows(y, pmax, h)
        if solve is None:
            phi = compressed_solution(sketch_rows(yy, h, idx, scale))
        else:
            phi = solve(yy, h, idx, scale)
        phis.append(phi)
        rows.append((idx, scale))
        tau[h - 1] = phi[h - 1]
    hit = np.nonzero(np.abs(tau) >= 1.96 / np.sqrt(c))[0]
    return {"tau": tau, "phi": phis, "rows": rows, "order": int(hit[-1] + 1) if hit.size else 0,
            "scores": kept}
