"""Pins for oracle.leverage (Definition 2.6, eq. (ldist), Section 3.1's p = 1
closed form, Definition 3.6 / eq. (glev), Theorem 3.7)."""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("p", [1, 2, 5, 9])
def test_scores_sum_to_d_and_nonnegative(p, rng):
    y = synth.ar_series(300, p, rng, 0.3, 0.9)
    X, _ = oracle.lag_matrix(y, p)
    l = oracle.leverage_scores(X)
    assert np.all(l >= -1e-15)
    assert abs(l.sum() - p) <= 1e-12 * p
    assert np.all(l <= 1 + 1e-12)


def test_hat_matrix_vs_qr_route(rng):
    y = synth.ar_series(120, 4, rng, 0.3, 0.9)
    X, _ = oracle.lag_matrix(y, 4)
    assert np.allclose(oracle.leverage_scores(X), oracle.leverage_scores_hat(X), atol=1e-13)


def test_p1_closed_form(rng):
    """Section 3.1: exact p = 1 scores are y_i^2 / sum_{t=1}^{n-1} y_t^2."""
    y = rng.standard_normal(200)
    X, _ = oracle.lag_matrix(y, 1)
    assert np.allclose(oracle.leverage_scores(X), oracle.ar1_leverage(y), rtol=1e-12, atol=0)


def test_generalized_wrt_self_is_leverage(rng):
    """Definition 3.6 with B = A gives the ordinary leverage scores."""
    y = synth.ar_series(200, 3, rng, 0.3, 0.9)
    X, _ = oracle.lag_matrix(y, 3)
    assert np.allclose(oracle.generalized_scores(X, X), oracle.leverage_scores(X), atol=1e-13)


def test_theorem_3_7_uniform_subsample_overestimates(rng):
    """Theorem 3.7: scores w.r.t. an (unscaled) uniform row subsample A_u are
    >= the true scores row by row; their expected total is <= n d / m'."""
    y = synth.ar_series(2000, 6, rng, 0.3, 0.9)
    X, _ = oracle.lag_matrix(y, 6)
    n, d = X.shape
    lev = oracle.leverage_scores(X)
    msub = 200
    totals = []
    for _ in range(40):
        idx = rng.choice(n, size=msub, replace=False)
        g = oracle.generalized_scores(X, X[idx])
        assert np.all(g >= lev * (1 - 1e-10))
        totals.append(g.sum())
    assert np.mean(totals) <= n * d / msub * 1.1


def test_glev_gform_equals_omega_form(rng):
    """eq. (glev): ||G B (B^T B)^{-1} C(i,:)||^2 equals the product form
    ||C(i,:)^T R_B^{-1} (G Q_B)^T||^2 with B = Q_B R_B (exact identity)."""
    y = synth.ar_series(400, 5, rng, 0.3, 0.9)
    X, _ = oracle.lag_matrix(y, 5)
    Bm = X[rng.choice(X.shape[0], 60, replace=True)] * 1.7
    G = rng.standard_normal((8, Bm.shape[0])) / np.sqrt(8)
    a = oracle.approx_generalized_scores(X, Bm, G)
    Q, R = np.linalg.qr(Bm)
    Pi = G @ Q
    Om = oracle.jl_omega(R, Pi)
    b = oracle.scores_from_omega(y, 5, Om)
    assert np.allclose(a, b, rtol=1e-10, atol=0)


def test_jl_scores_unbiased(rng):
    """E over Gaussian G (entries N(0,1/k)) of the eq. (glev) estimate equals
    the generalised score (Monte Carlo, 4 sigma)."""
    y = synth.ar_series(300, 4, rng, 0.3, 0.9)
    X, _ = oracle.lag_matrix(y, 4)
    Bm = X[::3]
    exact = oracle.generalized_scores(X, Bm)
    k, trials = 4, 3000
    acc = np.zeros_like(exact)
    for _ in range(trials):
        G = rng.standard_normal((k, Bm.shape[0])) / np.sqrt(k)
        acc += oracle.approx_generalized_scores(X, Bm, G)
    est = acc / trials
    # Var of chi^2_k / k scaled: 2/k * exact^2 per trial
    sd = np.sqrt(2.0 / k / trials) * exact
    assert np.all(np.abs(est - exact) <= 4.5 * sd + 1e-15)
