"""The five synthetic workloads, with their sizes, distributions and seeds.

Every workload is a deterministic function of its seed.  The paper's own
experiments use n = 2,000,000 samples of stationary AR(p) models with unit
innovation variance (Section 4.1); the sizes here follow the solver's target
configurations and stand in for data that is not available.

  ar3     AR(3), phi = (0.5, -0.3, 0.1), n = 10,000, N(0,1), burn-in 500,
          sketch 20p rows, tol 1e-10 (float64 path).
  ar100   AR(100), n = 2^22, 50 pole pairs, moduli U[0.5, 0.95], angles
          U(0, pi), N(0,1); sketch 8p rows, tol 1e-10 (float64 path).
  ar500   AR(500), n = 2^25, same pole generator (mixed-precision path).
  batch   2048 series, n = round(2^U(12,18)), p ~ U{4..64}, moduli
          U[0.3, 0.95], Student-t(5) innovations scaled to unit variance.
  serve   Poisson arrivals at 5000 fits/s; each request a series with
          n = round(2^U(10,20)), p ~ U{2..200}, moduli U[0.5, 0.95], N(0,1),
          drawn with replacement from a pre-generated pool.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .ar import ar_series, ar_series_direct, loguniform_length

AR3_PHI = (0.5, -0.3, 0.1)


@dataclass
class Fit:
    """One fitting problem: a series, its order, sketch multiplier and tolerance."""
    y: np.ndarray
    p: int
    gamma: int
    tol: float
    meta: dict = field(default_factory=dict)


def workload_ar3(seed: int = 0, n: int = 10_000) -> Fit:
    rng = np.random.default_rng(seed)
    y = ar_series_direct(n, AR3_PHI, rng, "normal", burn=500)
    return Fit(y, 3, 20, 1e-10, {"workload": "ar3", "n": n, "seed": seed})


def workload_ar100(seed: int = 0, n: int = 1 << 22) -> Fit:
    rng = np.random.default_rng(seed)
    y = ar_series(n, 100, rng, 0.5, 0.95, "normal")
    return Fit(y, 100, 8, 1e-10, {"workload": "ar100", "n": n, "seed": seed})


def workload_ar500(seed: int = 0, n: int = 1 << 25) -> Fit:
    rng = np.random.default_rng(seed)
    y = ar_series(n, 500, rng, 0.5, 0.95, "normal")
    return Fit(y, 500, 8, 1e-10, {"workload": "ar500", "n": n, "seed": seed})


def _batch_member(child: np.random.SeedSequence, lo_exp, hi_exp, p_lo, p_hi, r_lo, r_hi,
                  innovations) -> Fit:
    rng = np.random.default_rng(child)
    n = loguniform_length(rng, lo_exp, hi_exp)
    p = int(rng.integers(p_lo, p_hi + 1))
    y = ar_series(n, p, rng, r_lo, r_hi, innovations)
    return Fit(y, p, 8, 1e-10, {"n": n, "p": p})


def workload_batch(seed: int = 0, count: int = 2048, lo_exp: float = 12.0,
                   hi_exp: float = 18.0) -> list[Fit]:
    """Independent series for one batched launch (child seeds via SeedSequence.spawn)."""
    children = np.random.SeedSequence(seed).spawn(count)
    return [_batch_member(c, lo_exp, hi_exp, 4, 64, 0.3, 0.95, "t5") for c in children]


def workload_serve(seed: int = 0, rate: float = 5000.0, duration: float = 60.0,
                   pool: int = 4096, lo_exp: float = 10.0, hi_exp: float = 20.0):
    """(arrival_times_s, pool_index_per_request, pool_fits).

    Arrivals are a Poisson process (exponential inter-arrival times of mean
    1/rate); each request names a pool member drawn uniformly with
    replacement.  The pool holds `pool` series generated from spawned seeds.
    """
    ss = np.random.SeedSequence(seed)
    arr_ss, pool_ss = ss.spawn(2)
    rng = np.random.default_rng(arr_ss)
    expected = int(rate * duration * 1.2) + 16
    gaps = rng.exponential(1.0 / rate, expected)
    t = np.cumsum(gaps)
    t = t[t < duration]
    which = rng.integers(0, pool, t.size)
    children = pool_ss.spawn(pool)
    fits = [_batch_member(c, lo_exp, hi_exp, 2, 200, 0.5, 0.95, "normal") for c in children]
    for f in fits:
        f.tol = 1e-10
    return t, which, fits


def workload_pacf(seed: int = 0, n: int = 2_000_000) -> Fit:
    """AR(150), n = 2,000,000 (the size of the paper's PACF timing study,
    Section 4.1), pole generator with moduli U[0.5, 0.95]; PACF up to lag 250."""
    rng = np.random.default_rng(seed)
    y = ar_series(n, 150, rng, 0.5, 0.95, "normal")
    return Fit(y, 250, 8, 1e-10, {"workload": "pacf", "n": n, "seed": seed, "order": 150})


WORKLOADS = {
    "ar3": workload_ar3,
    "ar100": workload_ar100,
    "ar500": workload_ar500,
    "pacf": workload_pacf,
}
