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


def _rows_for(rng, R, c, pmax):
    out = []
    for _ in range(pmax):
        idx = rng.integers(0, R, c)
        out.append((idx, rng.uniform(0.5, 2.0, c)))
    return out


def test_pacf_compressed_all_rows_is_exact_pacf(rng):
    """Every row once at unit scale: the compressed estimate is the full
    least-squares fit, so the compressed PACF equals the exact one."""
    y = synth.ar_series(1500, 3, rng, 0.3, 0.9)
    pmax = 7
    R = y.size - pmax
    rows = [(np.arange(R), np.ones(R))] * pmax
    np.testing.assert_allclose(oracle.pacf_compressed(y, pmax, rows), oracle.pacf(y, pmax),
                               rtol=1e-11, atol=1e-14)


def test_pacf_compressed_lag1_closed_form(rng):
    """Lag 1 on sampled rows: the weighted one-column solution
    sum s^2 y[i] y[i+1] / sum s^2 y[i]^2 over the drawn rows i."""
    y = synth.ar_series(3000, 2, rng, 0.3, 0.9)
    pmax, c = 5, 200
    rows = _rows_for(rng, y.size - pmax, c, pmax)
    idx, s = rows[0]
    want = np.sum(s * s * y[idx] * y[idx + 1]) / np.sum(s * s * y[idx] ** 2)
    assert abs(oracle.pacf_compressed(y, pmax, rows)[0] - want) <= 1e-12 * abs(want)


def _fwl_sampled(y, h, idx, s):
    """Frisch-Waugh-Lovell on the weighted sampled rows with the lags taken by
    explicit indexing (response y[h+i], lag j value y[h+i-j]): the coefficient
    of y[t-h] in the weighted regression of y[t] on y[t-1..t-h]."""
    t = h + idx
    yt = s * y[t]
    xh = s * y[t - h]
    if h == 1:
        return np.dot(xh, yt) / np.dot(xh, xh)
    Z = np.column_stack([s * y[t - j] for j in range(1, h)])
    ey = yt - Z @ np.linalg.lstsq(Z, yt, rcond=None)[0]
    ex = xh - Z @ np.linalg.lstsq(Z, xh, rcond=None)[0]
    return np.dot(ex, ey) / np.dot(ex, ex)


def test_pacf_compressed_fwl_on_sampled_rows(rng):
    y = synth.ar_series(4000, 4, rng, 0.3, 0.9)
    pmax, c = 8, 300
    rows = _rows_for(rng, y.size - pmax, c, pmax)
    tau = oracle.pacf_compressed(y, pmax, rows)
    for h in range(1, pmax + 1):
        want = _fwl_sampled(y, h, *rows[h - 1])
        assert abs(tau[h - 1] - want) <= 1e-10 * max(1.0, abs(want)), h


def test_planted_window_slip_fails_the_pins(rng):
    """A compressed PACF that builds lag h's rows from the wrong window (one
    sample late, a plausible slip) fails the sampled-row pin."""
    y = synth.ar_series(4000, 4, rng, 0.3, 0.9)
    pmax, c = 6, 300
    rows = _rows_for(rng, y.size - pmax - 1, c, pmax)

    def slipped(y, pmax, rows):
        n = y.size
        return np.array([oracle.compressed_solution(
            oracle.sketch_rows(y[1: n - pmax + h + 1], h, *rows[h - 1]))[h - 1]
            for h in range(1, pmax + 1)])

    bad = slipped(y, pmax, rows)
    want = np.array([_fwl_sampled(y, h, *rows[h - 1]) for h in range(1, pmax + 1)])
    assert np.max(np.abs(bad - want)) > 1e-3
    np.testing.assert_allclose(oracle.pacf_compressed(y, pmax, rows), want, rtol=1e-9, atol=1e-12)
