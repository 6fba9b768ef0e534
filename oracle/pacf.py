"""Partial autocorrelations estimated through TOLS (oracle; test
infrastructure only).

Definition of the PACF: at lag h, the correlation of Y_t and Y_{t-h} after
the linear regression of both on the intermediate values.  Estimated through
the AR(h) least-squares fit (the paper's CMLE), tau_h is the fit's last
coefficient phi_{h,h} (by the Frisch-Waugh-Lovell theorem, the regression
coefficient of the residuals of y_t on the residuals of y_{t-h}).  As in
Algorithm 3, lag h uses the series prefix of n - pmax + h samples, so every
fit has n - pmax rows; the order estimate is the largest h with
|tau_h| >= 1.96 / sqrt(rows_h).

pacf calls fit_qr once per lag; pacf_compressed does the same with the
compressed estimator on given sampled rows.

Parity pins (tests/test_oracle_pacf.py): the h = 1 closed form
sum y_i y_{i+1} / sum y_i^2 over the rows; the Frisch-Waugh-Lovell ratio of
independently computed residuals (numpy lstsq) at every lag; an AR(1) series
whose PACF vanishes beyond lag 1 within its sampling band.  pacf_compressed:
with every row once at unit scale it equals pacf; its lag-1 value on sampled
rows has the weighted closed form sum s^2 y_i y_{i+1} / sum s^2 y_i^2; at
every lag it equals the weighted Frisch-Waugh-Lovell ratio on the sampled
rows with the lags taken by explicit indexing (a window one sample off fails
that pin, which a test plants and checks).
"""
from __future__ import annotations

import numpy as np

from .ols import fit_qr
from .sketch import compressed_solution, sketch_rows


def pacf(y, pmax: int) -> np.ndarray:
    """tau_1 .. tau_pmax (module doc)."""
    y = np.asarray(y, np.float64)
    n = y.size
    return np.array([fit_qr(y[: n - pmax + h], h)["phi"][h - 1] for h in range(1, pmax + 1)])


def pacf_compressed(y, pmax: int, rows) -> np.ndarray:
    """tau_h from the compressed estimator of lag h on rows[h-1] = (idx, scale)."""
    y = np.asarray(y, np.float64)
    n = y.size
    out = []
    for h in range(1, pmax + 1):
        idx, scale = rows[h - 1]
        out.append(compressed_solution(sketch_rows(y[: n - pmax + h], h, idx, scale))[h - 1])
    return np.array(out)


def pacf_order(tau, rows) -> int:
    """Largest h with |tau_h| >= 1.96 / sqrt(rows_h), 0 when none (Algorithm 3)."""
    tau = np.asarray(tau, np.float64)
    rows = np.broadcast_to(np.asarray(rows, np.float64), tau.shape)
    hit = np.nonzero(np.abs(tau) >= 1.96 / np.sqrt(rows))[0]
    return int(hit[-1] + 1) if hit.size else 0
