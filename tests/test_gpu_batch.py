"""Batched fits (tls_fit_batch, tls_fit_batch_device): every fit of a batch
equals the single fit with the same options and request id bit for bit, over
mixed lengths and orders that span several launch classes (FFT block length,
Cholesky and inverse tile counts, LDS staging of the step), with invalid and
degenerate fits mixed in; spot checks against the FP64 QR oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import capi, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = capi()
    with c.Context(0) as cx:
        yield cx


def _same_as_single(ctx, ys, ps, outs, rid0, device=False, **opts):
    for i, (y, p, o) in enumerate(zip(ys, ps, outs)):
        if device:
            single = ctx.fit_device(to_dev(y), p, 1e-10, request_id=rid0 + i, **opts)
        else:
            single = ctx.fit(y, p, 1e-10, request_id=rid0 + i, **opts)
        assert o["status"] == single["status"], (i, p, y.size)
        assert o["coef"].tobytes() == single["coef"].tobytes(), (i, p, y.size)
        if "iters" in o:
            assert o["iters"] == single["iters"], (i, p, y.size)
        if "resid_norm" in o:
            assert o["resid_norm"] == single["resid_norm"], (i, p, y.size)
        if "mixed_path" in o:
            assert o["mixed_path"] == single["mixed_path"], (i, p, y.size)


def _ok_or_stalled(s, outs):
    """Every fit converged, or stalled at the rounding level of the products
    (TLS_ESTALL, istop 5: some of these short t5 series are conditioned
    beyond FP64 resolution); the batch reports the first such status."""
    c = capi()
    for o in outs:
        assert o["status"] in (c.TLS_OK, c.TLS_ESTALL)
        assert (o["status"] == c.TLS_ESTALL) == (o["istop"] == 5)
    first = next((o["status"] for o in outs if o["status"] != c.TLS_OK), c.TLS_OK)
    assert s == first


def test_batch_host_equals_single(ctx):
    say("batch host")
    fits = synth.workload_batch(seed=11, count=24, lo_exp=12, hi_exp=15)
    ys, ps = [f.y for f in fits], [f.p for f in fits]
    s, outs = ctx.fit_batch(ys, ps, 1e-10, request_id=500)
    assert s == capi().TLS_OK
    _same_as_single(ctx, ys, ps, outs, 500)


def test_batch_device_equals_single(ctx):
    say("batch device")
    fits = synth.workload_batch(seed=12, count=32, lo_exp=12, hi_exp=16)
    ys, ps = [f.y for f in fits], [f.p for f in fits]
    s, outs = ctx.fit_batch_device([to_dev(y) for y in ys], ps, 1e-10, request_id=7)
    _ok_or_stalled(s, outs)
    say("   classes span B =", sorted({o["block_len"] for o in outs}))
    _same_as_single(ctx, ys, ps, outs, 7, device=True)


def test_batch_orders_across_kernel_limits(ctx):
    """p = 127, 128 (q = 129: the 32 x 32 register grid), 150 and 200 (no LDS
    staging of M), 250 and 300 (blocked Cholesky and inverse with different
    block counts), with small orders in the same batch."""
    say("batch wide orders")
    rng = np.random.default_rng(13)
    ps = [3, 127, 128, 150, 200, 16, 128, 250, 300, 260]
    ys = [synth.ar_series(int(n), p, rng, 0.3, 0.85)
          for n, p in zip([5000, 40000, 30000, 50000, 60000, 9000, 20000, 60000, 70000, 50000], ps)]
    s, outs = ctx.fit_batch_device([to_dev(y) for y in ys], ps, 1e-10, request_id=40)
    _ok_or_stalled(s, outs)
    _same_as_single(ctx, ys, ps, outs, 40, device=True)


def test_batch_wide_step_orders_equal_single(ctx):
    """Orders above 128 whose single fits take the wide LSQR step (the two
    products over many workgroups, four launches) while the batched step runs
    one workgroup per fit: both give the same bits, with FP64 products up to
    the batched kernels' largest order (623; 700 and 1024 run one at a time
    inside the call) and with FP32 products (mixed precision, path 1 on well
    conditioned series of orders just above 128)."""
    say("batch wide step orders")
    rng = np.random.default_rng(23)
    ps = [129, 623, 700, 1024]
    ys = [synth.ar_series(int(n), p, rng, 0.3, 0.8)
          for n, p in zip([20000, 30000, 30000, 40000], ps)]
    s, outs = ctx.fit_batch_device([to_dev(y) for y in ys], ps, 1e-10, request_id=60)
    _ok_or_stalled(s, outs)
    _same_as_single(ctx, ys, ps, outs, 60, device=True)
    # kappa_F >= q, so the FP32-product band (kappa_F <= 300) holds orders
    # just above 128 on nearly white series
    ps = [130, 140, 160]
    ys = [synth.ar_series(int(n), p, rng, 0.05, 0.2) for n, p in zip([30000, 50000, 60000], ps)]
    s, outs = ctx.fit_batch_device([to_dev(y) for y in ys], ps, 1e-10, request_id=70, precision=1)
    assert s in (capi().TLS_OK, capi().TLS_ENOCONV)
    paths = [o["mixed_path"] for o in outs]
    say("   paths", paths)
    assert 1 in paths
    _same_as_single(ctx, ys, ps, outs, 70, device=True, precision=1)


def test_batch_mixed_precision_equals_single(ctx):
    say("batch mixed")
    rng = np.random.default_rng(14)
    ps = [4, 20, 60, 33, 100]
    ys = [synth.ar_series(int(n), p, rng, 0.3, 0.85)
          for n, p in zip([8000, 30000, 70000, 20000, 50000], ps)]
    s, outs = ctx.fit_batch_device([to_dev(y) for y in ys], ps, 1e-10, request_id=3, precision=1)
    assert s in (capi().TLS_OK, capi().TLS_ENOCONV)
    say("   paths", [o["mixed_path"] for o in outs])
    _same_as_single(ctx, ys, ps, outs, 3, device=True, precision=1)


def test_batch_uniform_sketch_and_all_rows(ctx):
    """Uniform sketch, and short series whose sketch covers every row."""
    say("batch uniform / all rows")
    rng = np.random.default_rng(15)
    ps = [20, 6, 30, 10]
    ys = [synth.ar_series(int(n), p, rng, 0.3, 0.9) for n, p in zip([300, 40, 20000, 5000], ps)]
    for sketch in (0, 1):
        s, outs = ctx.fit_batch(ys, ps, 1e-10, request_id=90, sketch=sketch)
        assert s == capi().TLS_OK
        _same_as_single(ctx, ys, ps, outs, 90, sketch=sketch)


def test_batch_invalid_fits_reported_per_fit(ctx):
    c = capi()
    say("batch invalid")
    rng = np.random.default_rng(16)
    good = synth.ar_series(5000, 5, rng, 0.3, 0.9)
    bad = good.copy()
    bad[17] = np.inf
    const = np.full(3000, 1.5)
    ys = [good, bad, good[:8], const, good]
    ps = [5, 5, 5, 3, 5]
    s, outs = ctx.fit_batch(ys, ps, 1e-10, request_id=0)
    sts = [o["status"] for o in outs]
    say("   statuses", sts)
    assert sts[0] == c.TLS_OK and sts[4] == c.TLS_OK
    assert sts[1] == c.TLS_EINVAL
    assert sts[2] == c.TLS_EINVAL  # n < 2p + 1
    assert sts[3] == c.TLS_ERANK
    assert s == c.TLS_EINVAL
    single = ctx.fit(good, 5, 1e-10, request_id=4)
    assert outs[4]["coef"].tobytes() == single["coef"].tobytes()


def test_batch_empty(ctx):
    s, outs = ctx.fit_batch_device([], [], 1e-10)
    assert s == capi().TLS_OK and outs == []


def test_batch_against_oracle(ctx):
    """A few fits of a batch against the FP64 QR oracle (coefficient gate 1e-6
    on moderately conditioned series)."""
    say("batch vs oracle")
    rng = np.random.default_rng(17)
    ps = [2, 9, 31, 64]
    ys = [synth.ar_series(int(n), p, rng, 0.3, 0.8) for n, p in zip([3000, 12000, 40000, 90000], ps)]
    s, outs = ctx.fit_batch_device([to_dev(y) for y in ys], ps, 1e-10)
    assert s == capi().TLS_OK
    for y, p, o in zip(ys, ps, outs):
        ref = oracle.fit_qr(y, p)
        err = oracle.rel_error(o["coef"], ref["phi"])
        say("   p=%d kappa=%.3g err=%.3g" % (p, ref["kappa"], err))
        assert err <= 1e-6
        assert abs(o["resid_norm"] - ref["rnorm"]) <= 1e-9 * ref["rnorm"]


@pytest.mark.parametrize("max_refine", [0, 8])
def test_batch_mixed_paths_equal_single(ctx, max_refine):
    """Mixed batch with well and badly conditioned series together (pole
    moduli 0.3-0.85 and 0.5-0.95): each fit takes its own path (FP32-product
    LSQR, refinement when allowed, FP64 LSQR) inside the batch, bit for bit
    as alone, and reaches the FP64 path's residual."""
    say("batch mixed paths", max_refine)
    rng = np.random.default_rng(18)
    ps = [40, 64, 12, 50, 8, 30]
    mods = [(0.5, 0.95)] * 4 + [(0.3, 0.6)] * 2
    ys = [synth.ar_series(int(n), p, rng, *m)
          for n, p, m in zip([60000, 100000, 20000, 80000, 30000, 50000], ps, mods)]
    s, outs = ctx.fit_batch_device([to_dev(y) for y in ys], ps, 1e-10, request_id=9, precision=1,
                                   max_refine=max_refine)
    assert s == capi().TLS_OK
    _same_as_single(ctx, ys, ps, outs, 9, device=True, precision=1, max_refine=max_refine)
    paths = [o["mixed_path"] for o in outs]
    say("   paths", paths)
    assert 1 in paths and (3 if max_refine == 0 else 2) in paths
    for y, p, o in zip(ys, ps, outs):
        f64 = ctx.fit(y, p, 1e-10)
        say("   p=%d path=%d refine=%d iters=%d istop=%d resid %.12g vs %.12g"
            % (p, o["mixed_path"], o["refine_steps"], o["iters"], o["istop"], o["resid_norm"],
               f64["resid_norm"]))
        assert (o["refine_steps"] > 0) == (o["mixed_path"] == 2)
        assert abs(o["resid_norm"] - f64["resid_norm"]) <= 1e-9 * f64["resid_norm"]


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_graph_replay_equals_direct_launches(ctx, prec):
    """Each chunk of LSQR (or inner refinement) steps of a class is a HIP
    graph replayed many times; three calls in a row, with other device work
    and synchronisations between them, equal the directly launched batch bit
    for bit."""
    c = capi()
    say("batch graphs", prec)
    fits = synth.workload_batch(seed=19, count=40, lo_exp=12, hi_exp=16)
    ys, ps = [f.y for f in fits], [f.p for f in fits]
    devs = [to_dev(y) for y in ys]
    s0, ref = ctx.fit_batch_device(devs, ps, 1e-10, request_id=11, precision=prec, no_graph=1)
    for rep in range(3):
        ctx.fit(ys[rep], ps[rep], 1e-10)  # eager work between the replays
        s1, got = ctx.fit_batch_device(devs, ps, 1e-10, request_id=11, precision=prec)
        assert s1 == s0
        for a, b in zip(ref, got):
            assert a["status"] == b["status"]
            assert a["coef"].tobytes() == b["coef"].tobytes()
            assert a["iters"] == b["iters"]
