"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package draws random series and random numbers only.  It holds none of
the least-squares arithmetic: no lag matrices, no products, no factorisations.
"""
from .ar import (  # noqa: F401
    ar_series,
    ar_series_direct,
    sinusoid_series,
    add_outliers,
    loguniform_length,
    poles_to_coefficients,
    sinusoid_coefficients,
)
from .workloads import (  # noqa: F401
    workload_ar3,
    workload_ar100,
    workload_ar500,
    workload_batch,
    workload_serve,
    WORKLOADS,
)
