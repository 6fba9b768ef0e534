"""Repeated halving sketch (sketch = TLS_SKETCH_RH, Algorithm 4): the level
mask equals the oracle's nested halvings bit for bit; with a single level it
is the leverage sketch bit for bit; fits converge to the OLS solution like
the other sketches; the compressed estimate's residual ratio is in
[1, 1 + eps); batched calls equal single fits; servers reject it."""
import math

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


@pytest.mark.parametrize("p,n,seed", [(6, 60000, 0), (12, 150000, 1), (20, 400000, 2)])
def test_rh_compressed_matches_oracle(ctx, p, n, seed):
    """The compressed estimate from the repeated-halving sketch against the
    oracle's Algorithm 4 fed the same Philox draws (smallest level's uniform
    trials, the rows' level draws, the SRHT map, each level's leverage
    draws); both take every level's scores with respect to the factor of one
    shifted Cholesky QR sweep of the level below (oracle.shifted_r).  The
    factors differ by rounding, which moves no draw on these
    well-conditioned series, so the estimates agree to the QR backward error
    plus that rounding's effect on the row scales."""
    c = capi()
    say("rh compressed vs oracle", p, n)
    rng = np.random.default_rng(70 + seed)
    y = synth.ar_series(n, p, rng, 0.3, 0.7)
    fit_id, rseed, k = 5 + seed, 13, 8
    cc = 8 * p
    out = ctx.fit(y, p, 1e-10, sketch=c.SKETCH_RH, estimator=c.EST_SKETCH, seed=rseed,
                  request_id=fit_id)
    assert out["status"] == c.TLS_OK
    m = n - p
    levels = oracle.rh_levels(m, cc)
    P = 1 << max(0, math.ceil(math.log2(p)))
    Pi = oracle.srht_map(p, k, oracle.philox_uniform(P, c.RNG_SRHT_SIGNS, fit_id, rseed),
                         oracle.philox_uniform(k, c.RNG_SRHT_ROWS, fit_id, rseed))
    draws = [oracle.philox_uniform(cc, c.RNG_LEVERAGE, fit_id, rseed, start=i * cc)
             for i in range(levels)]
    A, idx, scale, lev = oracle.rh_sketch(
        y, p, cc, oracle.philox_uniform(cc, c.RNG_UNIFORM_ROWS, fit_id, rseed),
        oracle.philox_uniform(m, c.RNG_RH_LEVEL, fit_id, rseed), Pi, draws)
    assert lev == levels and levels >= 3
    ref = oracle.compressed_solution(A)
    kap = oracle.kappa(np.linalg.qr(A[:, :-1], mode="r"))
    err = oracle.rel_error(out["coef"], ref)
    shift_rel = 16 * (p + 1) * 2.0 ** -53 * kap ** 2
    say("   levels=%d kappa(SX)=%.3g err=%.3g" % (levels, kap, err))
    assert err <= max(1e-12, 1e-14 * kap * p) + 4 * kap * shift_rel
    assert abs(out["resid_norm"] - oracle.residual_norm(y, p, ref)) <= 1e-9 * out["resid_norm"]
