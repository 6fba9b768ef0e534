"""Seeded AR(p) series generators.

The process follows the autoregressive model of Section 3 (Definition of an
AR(p) model): Y_t = phi_1 Y_{t-1} + ... + phi_p Y_{t-p} + W_t with i.i.d.
zero-mean innovations.  Stationary coefficient sets are drawn through their
poles: p/2 complex-conjugate pairs r e^{+-i theta} with r inside the unit disc
(plus one real pole for odd p), so 1 - sum_j phi_j z^j = prod_k (1 - z/z_k)
has every root outside the unit circle.

The series is produced by a cascade of second-order recursive sections, one
per pole pair, in float64.  The cascade is the same linear filter 1/A(z) as
the direct-form recursion but stays numerically stable for large p, where the
direct-form coefficients reach 1e12 and amplify rounding.

Draw order (fixed, so a seed names one series): pole moduli for every pair,
then pair angles, then (odd p) the real pole's modulus and sign, then the
n + burn innovations.
"""
from __future__ import annotations

import numpy as np
from scipy.signal import lfilter, sosfilt

__all__ = [
    "ar_series",
    "ar_series_direct",
    "sinusoid_series",
    "add_outliers",
    "loguniform_length",
    "poles_to_coefficients",
    "sinusoid_coefficients",
]


def _innovations(rng: np.random.Generator, count: int, kind: str) -> np.ndarray:
    if kind == "normal":
        return rng.standard_normal(count)
    if kind == "t5":
        # Student-t with 5 degrees of freedom has variance 5/3; rescale to 1.
        return rng.standard_t(5, count) * np.sqrt(3.0 / 5.0)
    raise ValueError(f"unknown innovation kind {kind!r}")


def draw_poles(rng: np.random.Generator, p: int, r_lo: float, r_hi: float):
    """Pole moduli/angles for an order-p stationary AR model (see module doc)."""
    npairs = p // 2
    r = rng.uniform(r_lo, r_hi, npairs)
    theta = rng.uniform(0.0, np.pi, npairs)
    real_pole = None
    if p % 2:
        rr = rng.uniform(r_lo, r_hi)
        real_pole = rr if rng.random() < 0.5 else -rr
    return r, theta, real_pole


def _sections(r, theta, real_pole) -> np.ndarray:
    rows = [[1.0, 0.0, 0.0, 1.0, -2.0 * ri * np.cos(ti), ri * ri] for ri, ti in zip(r, theta)]
    if real_pole is not None:
        rows.append([1.0, 0.0, 0.0, 1.0, -float(real_pole), 0.0])
    return np.asarray(rows, dtype=np.float64).reshape(-1, 6)


def ar_series(n: int, p: int, rng: np.random.Generator, r_lo: float = 0.5,
              r_hi: float = 0.95, innovations: str = "normal", burn: int = 500,
              return_poles: bool = False):
    """n samples of a stationary AR(p) series from random poles (see module doc)."""
    if n < 1 or p < 1:
        raise ValueError("n and p must be positive")
    r, theta, real_pole = draw_poles(rng, p, r_lo, r_hi)
    x = _innovations(rng, n + burn, innovations)
    y = sosfilt(_sections(r, theta, real_pole), x)[burn:]
    y = np.ascontiguousarray(y, dtype=np.float64)
    if return_poles:
        return y, (r, theta, real_pole)
    return y


def ar_series_direct(n: int, phi, rng: np.random.Generator, innovations: str = "normal",
                     burn: int = 500) -> np.ndarray:
    """n samples of Y_t = sum_j phi_j Y_{t-j} + W_t by the direct recursion
    (zero initial state, the first `burn` samples discarded)."""
    phi = np.asarray(phi, dtype=np.float64)
    x = _innovations(rng, n + burn, innovations)
    a = np.concatenate(([1.0], -phi))
    return np.ascontiguousarray(lfilter([1.0], a, x)[burn:], dtype=np.float64)


def poles_to_coefficients(r, theta, real_pole) -> np.ndarray:
    """phi_1..phi_p of the AR model whose poles are given (sequential product
    of the real quadratic factors 1 - 2 r cos(theta) z + r^2 z^2)."""
    poly = np.array([1.0])
    for ri, ti in zip(r, theta):
        poly = np.convolve(poly, [1.0, -2.0 * ri * np.cos(ti), ri * ri])
    if real_pole is not None:
        poly = np.convolve(poly, [1.0, -float(real_pole)])
    return -poly[1:]


def sinusoid_series(n: int, freqs, amps, phases, const: float | None = None) -> np.ndarray:
    """Noise-free y_t = sum_k a_k cos(w_k t + psi_k) (+ const), t = 0..n-1.

    Each cosine satisfies y_t = 2 cos(w) y_{t-1} - y_{t-2} exactly and a
    constant satisfies y_t = y_{t-1}, so the sum obeys an AR recursion of
    order 2K (+1) with no innovation term."""
    t = np.arange(n, dtype=np.float64)
    y = np.zeros(n)
    for w, a, ps in zip(freqs, amps, phases):
        y += a * np.cos(w * t + ps)
    if const is not None:
        y += const
    return y


def sinusoid_coefficients(freqs, const: bool) -> np.ndarray:
    """phi of the exact recursion obeyed by sinusoid_series: the AR polynomial
    is prod_k (1 - 2 cos(w_k) z + z^2), times (1 - z) with a constant."""
    poly = np.array([1.0])
    for w in freqs:
        poly = np.convolve(poly, [1.0, -2.0 * np.cos(w), 1.0])
    if const:
        poly = np.convolve(poly, [1.0, -1.0])
    return -poly[1:]


def add_outliers(y: np.ndarray, rng: np.random.Generator, count: int) -> np.ndarray:
    """Outlier stress input (Section 4.2, synthetic data with outliers):
    `count` distinct positions are replaced by the value plus U[-3, 3] plus
    N(0, 100) noise.  Returns a new array."""
    out = np.array(y, dtype=np.float64, copy=True)
    idx = rng.choice(out.size, size=min(count, out.size), replace=False)
    out[idx] += rng.uniform(-3.0, 3.0, idx.size) + rng.normal(0.0, 10.0, idx.size)
    return out


def loguniform_length(rng: np.random.Generator, lo_exp: float, hi_exp: float) -> int:
    """round(2^U(lo_exp, hi_exp))."""
    return int(round(2.0 ** rng.uniform(lo_exp, hi_exp)))
