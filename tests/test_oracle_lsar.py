"""Pins of the LSAR oracle (Section 3.1: Definition of the approximate
leverage scores, eqs. (FALS), (FAR), (FASD); Algorithm 3)."""
import numpy as np
import pytest

import oracle
import synth
import oracle.lsar as L


def _exact_solve(yy, h, idx, scale):
    # the full least-squares solution of the lag, whatever rows were drawn
    return oracle.fit_qr(yy, h)["phi"]


def test_lag1_scores_are_definition_2_6(rng):
    y = synth.ar_series(700, 3, rng, 0.3, 0.9)
    pmax = 9
    X, _ = oracle.lag_matrix(L.lag_rows(y, pmax, 1), 1)
    np.testing.assert_allclose(L.scores_lag1(y, pmax), oracle.leverage_scores_hat(X),
                               rtol=1e-12, atol=0)


def test_recursion_with_exact_fits_gives_exact_leverage(rng):
    """eq. (FALS) with every lag's exact solution in place of the compressed
    one is the rank-one update of the hat matrix: the scores of every lag
    equal Definition 2.6 on that lag's lag matrix."""
    y = synth.ar_series(900, 4, rng, 0.3, 0.9)
    pmax, c = 7, 50
    draws = [rng.random(c) for _ in range(pmax)]
    out = L.lsar_pacf(y, pmax, c, draws, solve=_exact_solve, keep_scores=True)
    for h in range(1, pmax + 1):
        X, _ = oracle.lag_matrix(L.lag_rows(y, pmax, h), h)
        want = oracle.leverage_scores(X)
        np.testing.assert_allclose(out["scores"][h - 1], want, rtol=1e-9, atol=1e-15,
                                   err_msg=f"lag {h}")


def test_recursion_residual_indexing(rng):
    """eq. (FAR) row by row against the dense lag matrix of the lag's prefix."""
    y = rng.standard_normal(200)
    pmax = 6
    for h in range(1, pmax + 1):
        phi = rng.standard_normal(h)
        X, b = oracle.lag_matrix(L.lag_rows(y, pmax, h), h)
        np.testing.assert_allclose(L.residual(y, pmax, h, phi), X @ phi - b, rtol=0, atol=1e-13)


def test_scores_sum_to_lag(rng):
    """Each increment of eq. (FALS) sums to one: lag h's scores sum to h
    (eq. (FASD) is a distribution) whatever the coefficients."""
    y = synth.ar_series(3000, 5, rng, 0.3, 0.9)
    pmax, c = 12, 80
    draws = [rng.random(c) for _ in range(pmax)]
    out = L.lsar_pacf(y, pmax, c, draws, keep_scores=True)
    for h, s in enumerate(out["scores"], start=1):
        assert abs(s.sum() - h) <= 1e-11 * h
        assert np.all(s >= 0)


def test_tau_is_the_compressed_estimate_on_its_rows(rng):
    y = synth.ar_series(5000, 3, rng, 0.3, 0.9)
    pmax, c = 8, 120
    draws = [rng.random(c) for _ in range(pmax)]
    out = L.lsar_pacf(y, pmax, c, draws)
    tau = oracle.pacf_compressed(y, pmax, out["rows"])
    np.testing.assert_allclose(out["tau"], tau, rtol=1e-12, atol=1e-15)
    for h in range(1, pmax + 1):
        assert out["phi"][h - 1].size == h


def test_lsar_tracks_exact_pacf(rng):
    """With c well above the order, the compressed PACF of an AR(2) series
    follows the exact one within the sampling error, and the order rule
    finds the true order."""
    y = synth.ar_series_direct(200000, [0.5, -0.35], rng)
    pmax, c = 6, 4000
    draws = [rng.random(c) for _ in range(pmax)]
    out = L.lsar_pacf(y, pmax, c, draws)
    exact = oracle.pacf(y, pmax)
    assert np.max(np.abs(out["tau"] - exact)) <= 6 / np.sqrt(c)
    assert abs(out["tau"][1] + 0.35) <= 6 / np.sqrt(c)
    assert out["order"] >= 2


@pytest.mark.parametrize("shift", [1, -1])
def test_planted_row_shift_fails_the_exact_pin(rng, shift):
    """A residual taken one row off (a plausible indexing slip) breaks the
    exact-leverage pin: the pin catches it."""
    y = synth.ar_series(600, 3, rng, 0.3, 0.9)
    pmax = 5
    h = 3
    phi_prev = oracle.fit_qr(L.lag_rows(y, pmax, h - 1), h - 1)["phi"]
    good = L.scores_next(oracle.leverage_scores(oracle.lag_matrix(L.lag_rows(y, pmax, h - 1), h - 1)[0]),
                         L.residual(y, pmax, h - 1, phi_prev))
    r = np.roll(L.residual(y, pmax, h - 1, phi_prev), shift)
    bad = L.scores_next(oracle.leverage_scores(oracle.lag_matrix(L.lag_rows(y, pmax, h - 1), h - 1)[0]), r)
    want = oracle.leverage_scores(oracle.lag_matrix(L.lag_rows(y, pmax, h), h)[0])
    assert np.allclose(good, want, rtol=1e-9, atol=1e-15)
    assert not np.allclose(bad, want, rtol=1e-6, atol=1e-12)
