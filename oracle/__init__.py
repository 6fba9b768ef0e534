"""FP64 CPU oracle for the Toeplitz least-squares AR(p) fit.

TEST INFRASTRUCTURE ONLY.  This package is imported by tests/, by the
smoke() check in __graft_entry__.py and by the cpu_baseline leg of bench.py,
and by nothing else: the product library never imports, links or runs it.
It shares no code with the HIP path; the two meet only through the seeded
input generators in synth/.

Every function is a plain, slow, direct statement of what the paper defines
(dense lag matrix, dense products, LAPACK Householder QR, hat-matrix leverage
scores, inverse-CDF sampling), each citing its passage.

Parity status of each function is stated in its module header; the pins that
check it against mathematics other than itself live in tests/test_oracle_*.py.
"""
from .toeplitz import lag_matrix, matvec, rmatvec, block_windows, block_spectra  # noqa: F401
from .ols import (  # noqa: F401
    fit_qr, fit_svd, householder_qr, qr_r, kappa, rel_error, normal_residual,
    residual_norm, tri_inverse,
)
from .leverage import (  # noqa: F401
    leverage_scores, leverage_scores_hat, generalized_scores,
    approx_generalized_scores, scores_from_omega, ar1_leverage,
)
from .sketch import (  # noqa: F401
    uniform_rows, leverage_sample, sketch_rows, sketch_r, shifted_r, hadamard, srht_map,
    jl_omega,
    compressed_solution, rh_levels, rh_level_mask, rh_sketch,
)
from .philox import philox4x32_10, philox_uniform, philox_normal  # noqa: F401
from .lsqr import lsqr  # noqa: F401
from .pacf import pacf, pacf_compressed, pacf_order  # noqa: F401
from .lsar import lsar_pacf, scores_lag1, scores_next, residual as lsar_residual  # noqa: F401
