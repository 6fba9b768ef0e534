"""LSAR on the GPU (tls_lsar_device; Section 3.1, eqs. (FALS), (FAR), (FASD),
Algorithm 3) against the oracle.

The oracle replays Algorithm 3 lag by lag from the GPU's own coefficients of
the previous lag (so a draw that falls on the other side of a CDF boundary by
rounding cannot carry into later lags): at every lag its scores give the
sampled rows for the same Philox draws, which must match the GPU's rows except
at boundaries within rounding; its compressed solution on the GPU's rows must
match the GPU's coefficients within the backward error of a QR of that
sketch; and the last lag's scores must match the GPU's element by element
within the error of the FFT residual products.  Without replay, the oracle's
own lsar_pacf must give the same PACF and order."""
import math

import numpy as np
import pytest

import oracle
import oracle.lsar as olsar
import synth
from tests.gpu_common import EPS64, capi, fft_tol, say, to_dev, to_np, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = capi()
    with c.Context(0) as cx:
        yield cx


def _check_rows(scores, u, gi, c):
    """GPU rows vs the oracle's inverse-CDF rows for the same draws."""
    ri, _ = oracle.leverage_sample(scores, u, c)
    total = scores.sum()
    running = np.cumsum(scores)
    mism = np.nonzero(gi != ri)[0]
    for t in mism:  # only where the draw sits on a boundary within rounding
        assert abs(running[min(ri[t], gi[t])] - u[t] * total) <= 1e-11 * total, t
    assert np.all(scores[gi] > 0)
    return mism.size


# (generator order, n, pmax, c, seed, block_lg): several blocks with a ragged
# tail each; lag counts below, at and above the true order
CASES = [(3, 20000, 8, 120, 0, 0), (5, 60000, 24, 400, 1, 0), (12, 150000, 40, 800, 2, 9),
         (20, 250000, 70, 1000, 3, 0)]


@pytest.mark.parametrize("order_true,n,pmax,c,seed,block_lg", CASES)
def test_lsar_replay_matches_oracle(ctx, order_true, n, pmax, c, seed, block_lg):
    cap = capi()
    torch, dev = torch_dev()
    say("lsar replay", order_true, n, pmax, c, seed, block_lg)
    rng = np.random.default_rng(200 + seed)
    y = synth.ar_series(n, order_true, rng, 0.5, 0.9)
    R = n - pmax
    dscores = torch.zeros(R, dtype=torch.float64, device=dev)
    fit_id, rseed = 11 + seed, 5
    out = ctx.lsar_device(to_dev(y), pmax, c, d_scores=dscores, seed=rseed, request_id=fit_id,
                          block_lg=block_lg)
    assert out["status"] == cap.TLS_OK
    assert np.all(out["lag_status"] == cap.TLS_OK)
    B = (1 << block_lg) if block_lg else 1 << max(8, math.ceil(math.log2(8 * pmax)))
    scores, mism, err_bound = None, 0, np.zeros(R)
    for h in range(1, pmax + 1):
        if h == 1:
            r = -y[:R]
            scores = olsar.scores_lag1(y, pmax)
            v1 = 1.0
        else:
            phi_prev = out["phi"][h - 2]
            r = olsar.residual(y, pmax, h - 1, phi_prev)
            scores = olsar.scores_next(scores, r)
            v1 = 1.0 + np.abs(phi_prev).sum()
        # error of one increment r_i^2 / ||r||^2 when r comes from an FFT
        # product with elementwise error <= d (first order in d)
        d = fft_tol(EPS64, B, np.abs(y).max() * v1)
        rr = r @ r
        err_bound += (2 * np.abs(r) * d + d * d) / rr + (r * r / rr) * (2 * math.sqrt(R) * d
                                                                       / math.sqrt(rr))
        u = oracle.philox_uniform(c, cap.RNG_LEVERAGE, fit_id, rseed, start=(h - 1) * c)
        gi = out["rows"][h - 1]
        mism += _check_rows(scores, u, gi, c)
        # the compressed problem on the GPU's rows (scales from the scores)
        total = scores.sum()
        scale = 1.0 / np.sqrt(c * scores[gi] / total)
        A = oracle.sketch_rows(olsar.lag_rows(y, pmax, h), h, gi, scale)
        ref = oracle.compressed_solution(A)
        k = oracle.kappa(np.linalg.qr(A[:, :-1], mode="r"))
        err = oracle.rel_error(out["phi"][h - 1], ref)
        # QR backward error, plus the GPU's row scales 1/sqrt(c pi) differing
        # from these by half the scores' relative error
        srel = np.max(err_bound[gi] / scores[gi])
        assert err <= max(1e-12, 1e-14 * k * h) + 2 * k * srel, (h, err, k, srel)
        assert out["pacf"][h - 1] == out["phi"][h - 1][h - 1]
    say("   boundary mismatches %d of %d draws" % (mism, pmax * c))
    assert mism <= max(2, pmax * c // 5000)
    got = to_np(dscores)
    assert np.all(np.abs(got - scores) <= 4 * err_bound + 8 * EPS64 * pmax * scores)
    # Every increment sums to one: the scores of lag pmax sum to pmax (eq. (FASD))
    assert abs(got.sum() - pmax) <= 1e-9 * pmax
    # order rule on the returned PACF
    band = 1.96 / math.sqrt(c)
    hit = np.nonzero(np.abs(out["pacf"]) >= band)[0]
    assert out["order"] == (hit[-1] + 1 if hit.size else 0)


def test_lsar_matches_oracle_end_to_end(ctx):
    """No replay: the oracle's own Algorithm 3 from the same draws.  On a
    well-separated case no draw sits on a boundary, so the rows and the PACF
    agree exactly up to the compressed solves' rounding."""
    cap = capi()
    say("lsar end to end")
    rng = np.random.default_rng(31)
    n, pmax, c, fit_id, rseed = 40000, 16, 300, 3, 9
    y = synth.ar_series(n, 6, rng, 0.5, 0.9)
    out = ctx.lsar_device(to_dev(y), pmax, c, seed=rseed, request_id=fit_id)
    assert out["status"] == cap.TLS_OK
    draws = [oracle.philox_uniform(c, cap.RNG_LEVERAGE, fit_id, rseed, start=(h - 1) * c)
             for h in range(1, pmax + 1)]
    ref = olsar.lsar_pacf(y, pmax, c, draws)
    same = [np.array_equal(out["rows"][h], ref["rows"][h][0]) for h in range(pmax)]
    say("   lags with identical rows: %d of %d" % (sum(same), pmax))
    if all(same):
        assert np.allclose(out["pacf"], ref["tau"], rtol=1e-9, atol=1e-12)
        assert out["order"] == ref["order"]
    else:
        # a boundary draw changed a lag's rows; the lags before it agree
        first = same.index(False)
        assert np.allclose(out["pacf"][:first], ref["tau"][:first], rtol=1e-9, atol=1e-12)


def test_lsar_deterministic_and_validates(ctx):
    cap = capi()
    torch, dev = torch_dev()
    rng = np.random.default_rng(4)
    y = synth.ar_series(30000, 4, rng, 0.5, 0.9)
    dy = to_dev(y)
    a = ctx.lsar_device(dy, 10, 200, seed=1)
    b = ctx.lsar_device(dy, 10, 200, seed=1)
    assert a["pacf"].tobytes() == b["pacf"].tobytes()
    assert np.array_equal(a["rows"], b["rows"])
    other = ctx.lsar_device(dy, 10, 200, seed=2)
    assert not np.array_equal(a["rows"], other["rows"])
    # c must be at least pmax + 1 and at most the number of rows; n >= 2 pmax + 1
    assert ctx.lsar_device(dy, 10, 10)["status"] == cap.TLS_EINVAL
    assert ctx.lsar_device(dy, 10, 30000)["status"] == cap.TLS_EINVAL
    assert ctx.lsar_device(to_dev(y[:20]), 10, 11)["status"] == cap.TLS_EINVAL
