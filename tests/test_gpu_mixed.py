"""Mixed precision (FP32 spectra and sketch scores; FP64 QR, recurrences and
residual) against the FP64 QR oracle.  Each fit's path comes from
kappa_F = ||R||_F ||R^{-1}||_F of its sketch factor: LSQR with FP32 products
where kappa_F <= 300 (path 1), FP64 refinement around FP32 inner solves when
asked for (max_refine > 0, path 2), FP64 LSQR otherwise (path 3).  Coefficient
gate 1e-4 relative wherever the attainable accuracy allows it; path 1 is
checked against the FP32 products' bounds, the others against the FP64
ones, on coefficients, fitted values and residual at any conditioning."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import (EPS32, EPS64, attainable, capi, chunked_matvec_norms, resid_tol,
                              say, to_dev)

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
    path = out["mixed_path"]
    if path == 1:
        # FP32 products to max(tol, 1e-7): the bounds with eta = 16 eps_32
        # log2(B) + 1e-7 in place of the FP64 one (attainable() scaled)
        eta32 = 16 * EPS32 * math.log2(out["block_len"]) + max(tol, 1e-7)
        eta64 = 16 * EPS64 * math.log2(out["block_len"]) + tol
        coef_b, fit_b = attainable(phi, ref["rnorm"], ref["kappa"], smax, xphi,
                                   float(np.linalg.norm(y[p:])), p, out["block_len"], tol)
        coef_b, fit_b = coef_b * eta32 / eta64, fit_b * eta32 / eta64
    else:
        coef_b, fit_b = attainable(phi, ref["rnorm"], ref["kappa"], smax, xphi,
                                   float(np.linalg.norm(y[p:])), p, out["block_len"], tol)
    err = oracle.rel_error(out["coef"], phi)
    say("   kappa=%.3g path=%d err=%.3g (bound %.2g) fit=%.3g refine=%d iters=%d istop=%d"
        % (ref["kappa"], path, err, coef_b, xd / xphi, out["refine_steps"], out["iters"],
           out["istop"]))
    assert path in (1, 2, 3)
    if path == 1:
        # taken only where FP32 products meet the gate with a tenth to spare
        assert err <= gate / 10
    rt = resid_tol(phi, ref["rnorm"], smax, np.abs(y).max(), p, xd)
    if path == 1:
        # plus the second-order effect of the FP32 coefficients' own error
        rt = max(rt, 1.01 * xd * xd / (2 * ref["rnorm"]) + 1e-12 * ref["rnorm"])
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
    y = synth.ar_series(60000, 128, rng, 0.2, 0.6)
    out = ctx.fit(y, 128, 1e-10, precision=MIXED, block_lg=block_lg, max_refine=8)
    assert out["block_len"] == 1 << block_lg
    _check_mixed(out, y, 128)
    assert out["mixed_path"] == 2 and out["refine_steps"] >= 1


def test_mixed_ar500_shape(ctx):
    """AR(500) from the pole generator (moduli U[0.3, 0.8] to stay within
    FP32-resolvable conditioning), n = 2^16: exercises the p > 128 kernels."""
    say("mixed ar500")
    rng = np.random.default_rng(5)
    y = synth.ar_series(1 << 16, 500, rng, 0.3, 0.8)
    out = ctx.fit(y, 500, 1e-10, precision=MIXED)
    _check_mixed(out, y, 500)


def test_mixed_wide_step_fp32_products(ctx):
    """Order 140 on a nearly white series: kappa_F of the sketch factor is
    within the FP32-product band (kappa_F >= q), so the fit runs LSQR with
    FP32 products through the wide step (its products over many workgroups)
    and meets the FP32 products' bounds against the oracle."""
    say("mixed wide step fp32")
    rng = np.random.default_rng(29)
    y = synth.ar_series(60000, 140, rng, 0.05, 0.2)
    out = ctx.fit(y, 140, 1e-10, precision=MIXED)
    assert out["mixed_path"] == 1
    _check_mixed(out, y, 140)


def test_mixed_equals_f64_fitted_values(ctx):
    """Mixed and FP64 paths agree on a moderately conditioned AR(100) series."""
    say("mixed vs f64")
    rng = np.random.default_rng(7)
    y = synth.ar_series(1 << 18, 100, rng, 0.3, 0.85)
    a = ctx.fit(y, 100, 1e-10)
    b = ctx.fit(y, 100, 1e-10, precision=MIXED)
    xd, xphi = chunked_matvec_norms(y, 100, a["coef"] - b["coef"], a["coef"])
    say("   path %d fitted diff %.3g, resid %.12g vs %.12g"
        % (b["mixed_path"], xd / xphi, a["resid_norm"], b["resid_norm"]))
    assert a["status"] == capi().TLS_OK and b["status"] == capi().TLS_OK
    # FP32 products (path 1) resolve the fitted values to their own precision
    assert xd / xphi <= (1e-5 if b["mixed_path"] == 1 else 1e-9)
    assert abs(a["resid_norm"] - b["resid_norm"]) <= 1e-9 * a["resid_norm"]


def test_mixed_beyond_fp32_resolution_runs_fp64(ctx):
    """kappa(X) ~ 1e12 (the AR(100) pole workload) is beyond what FP32
    products resolve: the fit runs FP64 LSQR (path 3), also when refinement
    is allowed (its band ends at kappa_F = 1e8), and meets the FP64 bounds."""
    say("mixed beyond resolution")
    f = synth.workload_ar100(seed=0, n=1 << 18)
    a = ctx.fit(f.y, 100, 1e-10)
    for mr in (0, 8):
        b = ctx.fit(f.y, 100, 1e-10, precision=MIXED, max_refine=mr)
        say("   max_refine=%d path=%d istop=%d iters=%d resid %.12g vs %.12g" % (
            mr, b["mixed_path"], b["istop"], b["iters"], b["resid_norm"], a["resid_norm"]))
        assert b["mixed_path"] == 3 and b["refine_steps"] == 0 and b["istop"] in (1, 2)
        _check_mixed(b, f.y, 100)


def test_mixed_refinement_band(ctx):
    """max_refine > 0 and 300 < kappa_F <= 1e8: FP64 refinement around FP32
    inner solves (path 2), converging to the FP64 bounds; the same series
    without refinement runs FP64 LSQR (path 3)."""
    say("mixed refinement band")
    rng = np.random.default_rng(11)
    y = synth.ar_series(1 << 17, 40, rng, 0.5, 0.95)
    r = ctx.fit(y, 40, 1e-10, precision=MIXED, max_refine=8)
    d = ctx.fit(y, 40, 1e-10, precision=MIXED)
    say("   refine: path=%d refine=%d iters=%d; default: path=%d iters=%d"
        % (r["mixed_path"], r["refine_steps"], r["iters"], d["mixed_path"], d["iters"]))
    assert r["mixed_path"] == 2 and r["refine_steps"] >= 1
    assert d["mixed_path"] == 3 and d["refine_steps"] == 0
    _check_mixed(r, y, 40)
    _check_mixed(d, y, 40)


def test_mixed_device_input_deterministic(ctx):
    say("mixed determinism")
    rng = np.random.default_rng(6)
    y = synth.ar_series(50000, 20, rng, 0.3, 0.9)
    a = ctx.fit_device(to_dev(y), 20, 1e-10, precision=MIXED)
    b = ctx.fit(y, 20, 1e-10, precision=MIXED)
    assert a["coef"].tobytes() == b["coef"].tobytes()


def test_profiled_pass_kind(ctx):
    """profile = 1 reports which pass its timings cover: the fused FP64 pass
    for an FP64 fit and for a mixed fit that runs FP64 LSQR; the fused pass
    with FP32 products for a mixed fit on that path.  Profiling changes no
    result."""
    say("profiled pass kind")
    f = synth.workload_ar100(seed=0, n=1 << 18)
    a = ctx.fit(f.y, 100, 1e-10, profile=1)
    assert a["pass_kind"] == 0
    assert a["pass_count"] >= a["pass_worked"] >= a["iters"] >= 1 and a["pass_ms"] > 0
    b0 = ctx.fit(f.y, 100, 1e-10, precision=MIXED)
    b = ctx.fit(f.y, 100, 1e-10, precision=MIXED, profile=1)
    assert b["coef"].tobytes() == b0["coef"].tobytes()
    assert b["mixed_path"] == 3 and b["pass_kind"] == 0
    assert b["pass_count"] >= b["pass_worked"] >= 1 and b["pass_ms"] > 0
    g = synth.workload_ar3(seed=0)
    c0 = ctx.fit(g.y, 3, 1e-10, gamma=g.gamma, precision=MIXED)
    c = ctx.fit(g.y, 3, 1e-10, gamma=g.gamma, precision=MIXED, profile=1)
    say("   ar100 mixed kind=%d count=%d; ar3 mixed kind=%d path=%d istop=%d"
        % (b["pass_kind"], b["pass_count"], c["pass_kind"], c["mixed_path"], c["istop"]))
    assert c["coef"].tobytes() == c0["coef"].tobytes()
    assert c["mixed_path"] == 1 and c["pass_kind"] == 2 and c["pass_count"] >= c["pass_worked"] >= 1
