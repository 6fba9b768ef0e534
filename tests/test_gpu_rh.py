"""Repeated halving sketch (sketch = TLS_SKETCH_RH, Algorithm 4): the level
mask equals the oracle's nested halvings bit for bit; with a single level it
is the leverage sketch bit for bit; fits converge to the OLS solution like
the other sketches; the compressed estimate's residual ratio is in
[1, 1 + eps); batched calls equal single fits; servers reject it."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import capi, say, to_dev, to_np, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = capi()
    with c.Context(0) as cx:
        yield cx


@pytest.mark.parametrize("prec", [0, 1])
def test_rh_mask_matches_oracle(ctx, prec):
    c = capi()
    torch, dev = torch_dev()
    m, seed, fit = 200003, 9, 4
    u = oracle.philox_uniform(m, c.RNG_RH_LEVEL, fit, seed)
    for level in (0, 1, 3, 7):
        dt = torch.float64 if prec == 0 else torch.float32
        s = torch.ones(m, dtype=dt, device=dev)
        assert ctx.op_rh_mask(prec, s, m, level, seed, fit) == c.TLS_OK
        got = to_np(s) != 0
        assert np.array_equal(got, oracle.rh_level_mask(u, level)), level


def test_rh_single_level_is_leverage(ctx):
    """m <= 2c: one halving reaches c rows, so RH is the leverage sketch."""
    c = capi()
    rng = np.random.default_rng(30)
    y = synth.ar_series(1500, 100, rng, 0.3, 0.8)  # m = 1400 <= 2 * 800
    assert oracle.rh_levels(1400, 800) == 1
    for est in (c.EST_OLS, c.EST_SKETCH):
        a = ctx.fit(y, 100, 1e-10, sketch=c.SKETCH_RH, estimator=est)
        b = ctx.fit(y, 100, 1e-10, sketch=c.SKETCH_LEVERAGE, estimator=est)
        assert a["coef"].tobytes() == b["coef"].tobytes() and a["iters"] == b["iters"]


@pytest.mark.parametrize("p,n,seed", [(8, 100000, 0), (30, 300000, 1), (64, 1 << 20, 2)])
def test_rh_fit_matches_oracle(ctx, p, n, seed):
    c = capi()
    say("rh fit", p, n)
    rng = np.random.default_rng(40 + seed)
    y = synth.ar_series(n, p, rng, 0.3, 0.8)
    out = ctx.fit(y, p, 1e-10, sketch=c.SKETCH_RH)
    ref = oracle.fit_qr(y, p)
    err = oracle.rel_error(out["coef"], ref["phi"])
    levels = oracle.rh_levels(n - p, 8 * p)
    say("   levels=%d iters=%d kappa=%.3g err=%.3g" % (levels, out["iters"], ref["kappa"], err))
    assert out["status"] == c.TLS_OK and levels >= 3
    assert err <= 1e-8
    assert abs(out["resid_norm"] - ref["rnorm"]) <= 1e-9 * ref["rnorm"]
    lev = ctx.fit(y, p, 1e-10)
    assert out["iters"] <= 2 * lev["iters"] + 5  # a preconditioner of the same quality


def test_rh_compressed_ratio_batch_and_server(ctx):
    c = capi()
    say("rh compressed")
    rng = np.random.default_rng(50)
    ys = [synth.ar_series(n, p, rng, 0.3, 0.9) for n, p in [(80000, 10), (200000, 25)]]
    ps = [10, 25]
    for y, p in zip(ys, ps):
        comp = ctx.fit(y, p, 1e-10, sketch=c.SKETCH_RH, estimator=c.EST_SKETCH)
        ols = ctx.fit(y, p, 1e-10)
        ratio = comp["resid_norm"] / ols["resid_norm"]
        say("   p=%d residual ratio %.6f" % (p, ratio))
        assert comp["status"] == c.TLS_OK and 1.0 - 1e-12 <= ratio <= 1.5
    s, outs = ctx.fit_batch_device([to_dev(y) for y in ys], ps, 1e-10, sketch=c.SKETCH_RH,
                                   request_id=3)
    assert s == c.TLS_OK
    for i, (y, p) in enumerate(zip(ys, ps)):
        single = ctx.fit(y, p, 1e-10, sketch=c.SKETCH_RH, request_id=3 + i)
        assert outs[i]["coef"].tobytes() == single["coef"].tobytes()
    with pytest.raises(c.TlsError) as e:
        c.Server(ctx, 1 << 28, 8, sketch=c.SKETCH_RH)
    assert e.value.status == c.TLS_EUNSUPPORTED
