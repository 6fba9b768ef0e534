"""Mixed-precision path (FP32 FFT products and sketch scores; FP64 QR,
recurrences, residual and outer refinement, with an FP64 LSQR finish when
the FP32 products stop contracting) against the FP64 QR oracle.  Coefficient
gate 1e-4 relative wherever the attainable accuracy allows it, and the FP64
bounds on coefficients, fitted values and residual at any conditioning."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import attainable, capi, chunked_matvec_norms, resid_tol, say, to_dev

pytestmark = pytest.mark.gpu

MIXED = 1


@pytest.fixture(scope="module")
def ctx():
    c = capi()
    with c.Context(0) as cx:
        yield cx


def _check_mixed(out, y, p, gate=1e-4, tol=1e-10):
    c = capi()
    ref = oracle.fit_qr(y, p)
    phi = ref["phi"]
    smax = float(np.linalg.svd(ref["R"], compute_uv=False)[0])
    xd, xphi = chunked_matvec_norms(y, p, out["coef"] - phi, phi)
    coef_b, fit_b = attainable(phi, ref["rnorm"], ref["kappa"], smax, xphi,
                               float(np.linalg.norm(y[p:])), p, out["block_len"], tol)
    err = oracle.rel_error(out["coef"], phi)
    say("   kappa=%.3g err=%.3g (bound %.2g) fit=%.3g refine=%d inner=%d istop=%d"
        % (ref["kappa"], err, coef_b, xd / xphi, out["refine_steps"], out["iters"], out["istop"]))
    rt = resid_tol(phi, ref["rnorm"], smax, np.abs(y).max(), p, xd)
    if out["status"] == c.TLS_ESTALL:
        # the FP64 finish reached the rounding of its products before tol
        assert out["istop"] == 5 and coef_b > gate, (coef_b, out["istop"])
    else:
        assert out["status"] == c.TLS_OK, c.status_string(out["status"])
    if coef_b < gate:
        assert err <= gate
    assert err <= max(100 * coef_b, 1e-12)
    assert xd / xphi <= max(10 * fit_b, 1e-14)
    # the reported residual is the row-wise FP64 norm of the returned phi
    assert abs(out["resid_norm"] - ref["rnorm"]) <= rt
    return err


@pytest.mark.parametrize("p,n,seed,rlo,rhi", [(3, 10000, 0, 0.3, 0.9), (10, 65536, 1, 0.3, 0.9),
                                              (64, 131072, 2, 0.3, 0.9), (100, 65536, 3, 0.3, 0.85),
                                              (200, 100000, 4, 0.3, 0.8)])
def test_mixed_matches_oracle(ctx, p, n, seed, rlo, rhi):
    say("mixed", p, n, seed)
    rng = np.random.default_rng(seed)
    y = synth.ar_series(n, p, rng, rlo, rhi)
    out = ctx.fit(y, p, 1e-10, precision=MIXED)
    _check_mixed(out, y, p)


@pytest.mark.parametrize("block_lg", [12, 13, 14])
def test_mixed_p128_long_blocks(ctx, block_lg):
    """p = 128 with transform lengths 2^12..2^14: the refinement kernels'
    transform buffer leaves too little LDS for M there at the longer lengths,
    so they read M from global memory (the launch must not exceed LDS)."""
    say("mixed p128 block_lg", block_lg)
    rng = np.random.default_rng(40 + block_lg)
    y = synth.ar_series(60000, 128, rng, 0.3, 0.8)
    out = ctx.fit(y, 128, 1e-10, precision=MIXED, block_lg=block_lg)
    assert out["block_len"] == 1 << block_lg
    _check_mixed(out, y, 128)


def test_mixed_ar500_shape(ctx):
    """AR(500) from the pole generator (moduli U[0.3, 0.8] to stay within
    FP32-resolvable conditioning), n = 2^16: exercises the p > 128 kernels."""
    say("mixed ar500")
    rng = np.random.default_rng(5)
    y = synth.ar_series(1 << 16, 500, rng, 0.3, 0.8)
    out = ctx.fit(y, 500, 1e-10, precision=MIXED)
    _check_mixed(out, y, 500)


def test_mixed_equals_f64_fitted_values(ctx):
    """Mixed and FP64 paths agree on a moderately conditioned AR(100) series."""
    say("mixed vs f64")
    rng = np.random.default_rng(7)
    y = synth.ar_series(1 << 18, 100, rng, 0.3, 0.85)
    a = ctx.fit(y, 100, 1e-10)
    b = ctx.fit(y, 100, 1e-10, precision=MIXED)
    xd, xphi = chunked_matvec_norms(y, 100, a["coef"] - b["coef"], a["coef"])
    say("   fitted diff %.3g, resid %.12g vs %.12g" % (xd / xphi, a["resid_norm"], b["resid_norm"]))
    assert a["status"] == capi().TLS_OK and b["status"] == capi().TLS_OK
    assert xd / xphi <= 1e-9
    assert abs(a["resid_norm"] - b["resid_norm"]) <= 1e-9 * a["resid_norm"]


def test_mixed_beyond_fp32_resolution_finishes_in_fp64(ctx):
    """kappa(X) ~ 1e12 (the AR(100) pole workload) is beyond what FP32
    products resolve: the refinement stops contracting, FP64 LSQR finishes
    from its best iterate, and the result meets the FP64 bounds."""
    say("mixed beyond resolution")
    f = synth.workload_ar100(seed=0, n=1 << 18)
    a = ctx.fit(f.y, 100, 1e-10)
    b = ctx.fit(f.y, 100, 1e-10, precision=MIXED)
    say("   istop=%d refine=%d iters=%d resid %.12g vs %.12g" % (
        b["istop"], b["refine_steps"], b["iters"], b["resid_norm"], a["resid_norm"]))
    assert b["istop"] in (1, 2)
    _check_mixed(b, f.y, 100)


def test_mixed_device_input_deterministic(ctx):
    say("mixed determinism")
    rng = np.random.default_rng(6)
    y = synth.ar_series(50000, 20, rng, 0.3, 0.9)
    a = ctx.fit_device(to_dev(y), 20, 1e-10, precision=MIXED)
    b = ctx.fit(y, 20, 1e-10, precision=MIXED)
    assert a["coef"].tobytes() == b["coef"].tobytes()


def test_profiled_pass_kind(ctx):
    """profile = 1 reports which pass its timings cover: the fused FP64 pass
    for an FP64 fit; the FP32 normal-equation pass for a mixed fit whose
    refinement converges; for a mixed fit with an FP64 finish, whichever took
    more device time.  Profiling changes no result."""
    say("profiled pass kind")
    f = synth.workload_ar100(seed=0, n=1 << 18)
    a = ctx.fit(f.y, 100, 1e-10, profile=1)
    assert a["pass_kind"] == 0
    assert a["pass_count"] >= a["pass_worked"] >= a["iters"] >= 1 and a["pass_ms"] > 0
    b0 = ctx.fit(f.y, 100, 1e-10, precision=MIXED)
    b = ctx.fit(f.y, 100, 1e-10, precision=MIXED, profile=1)
    assert b["coef"].tobytes() == b0["coef"].tobytes()
    assert b["pass_kind"] in (0, 1) and b["pass_count"] >= b["pass_worked"] >= 1 and b["pass_ms"] > 0
    g = synth.workload_ar3(seed=0)
    c0 = ctx.fit(g.y, 3, 1e-10, gamma=g.gamma, precision=MIXED)
    c = ctx.fit(g.y, 3, 1e-10, gamma=g.gamma, precision=MIXED, profile=1)
    say("   ar100 mixed kind=%d count=%d; ar3 mixed kind=%d istop=%d refine=%d"
        % (b["pass_kind"], b["pass_count"], c["pass_kind"], c["istop"], c["refine_steps"]))
    assert c["coef"].tobytes() == c0["coef"].tobytes()
    assert c["pass_kind"] == 1 and c["pass_count"] >= c["pass_worked"] >= 1
