"""The compressed (sketch-and-solve) estimator, estimator = TLS_EST_SKETCH
(Section 2.1, eq. (OLSc)): with the uniform sketch its rows are reproducible,
so the GPU estimate is compared with the oracle's compressed solution on the
same rows; with the leverage sketch its residual ratio against the OLS fit
lies in [1, 1 + eps); with every row sampled it is the OLS solution; batched
and served fits equal the single fit bit for bit."""
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


@pytest.mark.parametrize("p,n,gamma,seed", [(4, 20000, 8, 0), (17, 60000, 8, 1), (40, 100000, 16, 2)])
def test_compressed_uniform_matches_oracle(ctx, p, n, gamma, seed):
    c = capi()
    say("compressed uniform", p, n, gamma)
    rng = np.random.default_rng(100 + seed)
    y = synth.ar_series(n, p, rng, 0.3, 0.8)
    rid = 7 + seed
    out = ctx.fit(y, p, 1e-10, estimator=c.EST_SKETCH, sketch=c.SKETCH_UNIFORM, gamma=gamma,
                  request_id=rid, seed=3)
    assert out["status"] == c.TLS_OK and out["iters"] == 0
    m, cc = n - p, gamma * p
    ri, rs = oracle.uniform_rows(oracle.philox_uniform(cc, c.RNG_UNIFORM_ROWS, rid, 3), m, cc)
    A = oracle.sketch_rows(y, p, ri, rs)
    ref = oracle.compressed_solution(A)
    k = oracle.kappa(np.linalg.qr(A[:, :-1], mode="r"))
    err = oracle.rel_error(out["coef"], ref)
    say("   kappa(SX)=%.3g err=%.3g" % (k, err))
    # backward-stable QR of the same rows: error <= c u kappa(SX) (generous c)
    assert err <= max(1e-12, 1e-14 * k * p)
    assert abs(out["resid_norm"] - oracle.residual_norm(y, p, ref)) <= 1e-9 * out["resid_norm"]


def test_compressed_leverage_residual_ratio(ctx):
    """The OLS residual is the smallest (ratio >= 1); the compressed one
    approaches it as the sketch grows (ratio at 64p below the one at 8p, and
    1 + eps with eps of the order of p / c)."""
    c = capi()
    say("compressed leverage")
    rng = np.random.default_rng(7)
    for p, n in [(10, 50000), (30, 120000)]:
        y = synth.ar_series(n, p, rng, 0.3, 0.9)
        ols = ctx.fit(y, p, 1e-10)
        ratios = {}
        for gamma in (8, 64):
            comp = ctx.fit(y, p, 1e-10, estimator=c.EST_SKETCH, gamma=gamma)
            assert comp["status"] == c.TLS_OK and comp["iters"] == 0
            ratios[gamma] = comp["resid_norm"] / ols["resid_norm"]
            say("   p=%d gamma=%d residual ratio %.6f coef err vs OLS %.3g"
                % (p, gamma, ratios[gamma], oracle.rel_error(comp["coef"], ols["coef"])))
            assert 1.0 - 1e-12 <= ratios[gamma] <= 1.5
        assert ratios[64] < ratios[8]
        # deterministic: the same call gives the same estimate
        again = ctx.fit(y, p, 1e-10, estimator=c.EST_SKETCH, gamma=64)
        assert np.array_equal(again["coef"], comp["coef"])


def test_compressed_all_rows_is_ols(ctx):
    c = capi()
    rng = np.random.default_rng(8)
    y = synth.ar_series(100, 12, rng, 0.3, 0.8)  # m = 88 <= c = 96: every row
    out = ctx.fit(y, 12, 1e-10, estimator=c.EST_SKETCH)
    ref = oracle.fit_qr(y, 12)
    assert out["status"] == c.TLS_OK
    assert oracle.rel_error(out["coef"], ref["phi"]) <= 1e-12 * max(1.0, ref["kappa"])


@pytest.mark.parametrize("prec", [0, 1])
def test_compressed_batch_and_serve_equal_single(ctx, prec):
    c = capi()
    say("compressed batch/serve", prec)
    fits = synth.workload_batch(seed=21, count=24, lo_exp=11, hi_exp=16)
    ys, ps = [f.y for f in fits], [f.p for f in fits]
    s, outs = ctx.fit_batch_device([to_dev(y) for y in ys], ps, 1e-10, request_id=40,
                                   estimator=c.EST_SKETCH, precision=prec)
    assert s == c.TLS_OK
    for i, (y, p, o) in enumerate(zip(ys, ps, outs)):
        single = ctx.fit(y, p, 1e-10, request_id=40 + i, estimator=c.EST_SKETCH, precision=prec)
        assert o["coef"].tobytes() == single["coef"].tobytes(), i
        assert o["resid_norm"] == single["resid_norm"] and o["iters"] == 0
    if prec == 0:
        with c.Server(ctx, 1 << 30, 64, estimator=c.EST_SKETCH) as srv:
            tickets = [srv.submit_device(to_dev(y), p, 1e-10, request_id=40 + i)
                       for i, (y, p) in enumerate(zip(ys, ps))]
            got = [srv.wait(t) for t in tickets]
        for o, g in zip(outs, got):
            assert o["coef"].tobytes() == g["coef"].tobytes()
            assert o["resid_norm"] == g["resid_norm"]


def test_estimator_rejects_unknown(ctx):
    c = capi()
    y = np.random.default_rng(0).standard_normal(1000)
    assert ctx.fit(y, 3, 1e-10, estimator=2)["status"] == c.TLS_EINVAL


@pytest.mark.parametrize("p,n,seed", [(6, 60000, 0), (15, 150000, 1), (40, 300000, 2)])
def test_compressed_leverage_matches_oracle(ctx, p, n, seed):
    """The one-level leverage sketch end to end against the oracle fed the
    same Philox draws: uniform trials -> R of one shifted Cholesky QR sweep
    (oracle.shifted_r) -> Omega = R^{-1} Pi^T with the SRHT map -> eq. (glev)
    scores -> leverage draws -> compressed solution.  The two factors differ
    by rounding (relative ~ q u kappa^2 of the uniform sketch), which moves
    no draw here, so the estimates agree to the final QR's backward error
    plus that rounding's effect on the row scales."""
    import math
    c = capi()
    say("compressed leverage vs oracle", p, n)
    rng = np.random.default_rng(90 + seed)
    y = synth.ar_series(n, p, rng, 0.3, 0.7)
    fit_id, rseed, k, cc = 21 + seed, 17, 8, 8 * p
    out = ctx.fit(y, p, 1e-10, estimator=c.EST_SKETCH, seed=rseed, request_id=fit_id)
    assert out["status"] == c.TLS_OK
    m = n - p
    P = 1 << max(0, math.ceil(math.log2(p)))
    Pi = oracle.srht_map(p, k, oracle.philox_uniform(P, c.RNG_SRHT_SIGNS, fit_id, rseed),
                         oracle.philox_uniform(k, c.RNG_SRHT_ROWS, fit_id, rseed))
    i0, s0 = oracle.uniform_rows(oracle.philox_uniform(cc, c.RNG_UNIFORM_ROWS, fit_id, rseed),
                                 m, cc)
    B = oracle.sketch_rows(y, p, i0, s0)
    sc = oracle.scores_from_omega(y, p, oracle.jl_omega(oracle.shifted_r(B, p), Pi))
    i1, s1 = oracle.leverage_sample(sc, oracle.philox_uniform(cc, c.RNG_LEVERAGE, fit_id, rseed),
                                    cc)
    A = oracle.sketch_rows(y, p, i1, s1)
    ref = oracle.compressed_solution(A)
    kap = oracle.kappa(np.linalg.qr(A[:, :-1], mode="r"))
    kap0 = oracle.kappa(np.linalg.qr(B[:, :p], mode="r"))
    r_rel = 16 * (p + 1) * 2.0 ** -53 * kap0 ** 2
    err = oracle.rel_error(out["coef"], ref)
    say("   kappa(SX)=%.3g err=%.3g" % (kap, err))
    assert err <= max(1e-12, 1e-14 * kap * p) + 4 * kap * r_rel
