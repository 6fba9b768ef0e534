"""Pins of the oracle's PACF (Definition of the PACF estimated through TOLS,
Algorithm 3's lag windows)."""
import numpy as np

import oracle
import synth


def test_pacf_lag1_closed_form(rng):
    y = synth.ar_series(3000, 4, rng, 0.3, 0.9)
    pmax = 6
    m = y.size - pmax
    x, b = y[:m], y[1:m + 1]  # lag 1 on the prefix of m + 1 samples
    want = np.dot(x, b) / np.dot(x, x)
    assert abs(oracle.pacf(y, pmax)[0] - want) <= 1e-13 * abs(want)


def test_pacf_frisch_waugh_lovell(rng):
    """tau_h = (e_x . e_y) / (e_x . e_x): e_y, e_x the residuals of y_t and
    y_{t-h} regressed (numpy lstsq) on y_{t-1} .. y_{t-h+1}."""
    y = synth.ar_series(2000, 5, rng, 0.3, 0.9)
    pmax = 8
    n = y.size
    tau = oracle.pacf(y, pmax)
    for h in range(2, pmax + 1):
        yy = y[: n - pmax + h]
        t = np.arange(h, yy.size)  # responses y_t, t = h .. len - 1
        Z = np.column_stack([yy[t - j] for j in range(1, h)])
        ey = yy[t] - Z @ np.linalg.lstsq(Z, yy[t], rcond=None)[0]
        ex = yy[t - h] - Z @ np.linalg.lstsq(Z, yy[t - h], rcond=None)[0]
        want = np.dot(ex, ey) / np.dot(ex, ex)
        assert abs(tau[h - 1] - want) <= 1e-10 * max(1.0, abs(want)), h


def test_pacf_ar1_cuts_off(rng):
    """AR(1), phi = 0.6: tau_1 near 0.6, later lags inside the 95% band
    (a few excursions allowed), order estimate 1 for this seed."""
    y = synth.ar_series_direct(40000, [0.6], rng)
    pmax = 10
    tau = oracle.pacf(y, pmax)
    band = 1.96 / np.sqrt(y.size - pmax)
    assert abs(tau[0] - 0.6) <= 4 / np.sqrt(y.size)
    assert np.sum(np.abs(tau[1:]) >= band) <= 2
    assert np.all(np.abs(tau[1:]) <= 2.5 * band)


def test_pacf_order_rule():
    tau = np.array([0.5, -0.2, 0.01, 0.03, 0.001])
    assert oracle.pacf_order(tau, 10000) == 4  # 0.03 >= 0.0196
    assert oracle.pacf_order(tau, 100) == 2    # band 0.196
    assert oracle.pacf_order(np.zeros(3), 50) == 0
