"""Partial autocorrelations (tls_pacf_device): exact PACF against the oracle
(one AR(h) least-squares fit per lag on Algorithm 3's windows), the
compressed PACF with the uniform sketch against the oracle's compressed
solutions on the same Philox rows, the order rule, argument errors."""
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


@pytest.mark.parametrize("p,pmax,n,seed", [(6, 16, 20000, 0), (3, 40, 50000, 1)])
def test_pacf_exact_matches_oracle(ctx, p, pmax, n, seed):
    c = capi()
    say("pacf exact", p, pmax, n)
    rng = np.random.default_rng(200 + seed)
    y = synth.ar_series(n, p, rng, 0.3, 0.8)
    s, tau, order, st = ctx.pacf_device(to_dev(y), pmax, 1e-12)
    assert s == c.TLS_OK and np.all(st == c.TLS_OK)
    ref = oracle.pacf(y, pmax)
    rows = n - pmax
    err = np.abs(tau - ref).max()
    say("   max |tau - oracle| = %.3g, order %d (oracle %d)"
        % (err, order, oracle.pacf_order(ref, rows)))
    assert err <= 1e-9
    band = 1.96 / np.sqrt(rows)
    if np.all(np.abs(np.abs(ref) - band) > 1e-6):  # no lag on the band's edge
        assert order == oracle.pacf_order(ref, rows)
    assert order >= p  # the true order's lag is far outside the band


def test_pacf_compressed_uniform_matches_oracle(ctx):
    c = capi()
    say("pacf compressed")
    rng = np.random.default_rng(210)
    n, p, pmax, gamma, seed, rid = 30000, 5, 12, 16, 4, 100
    y = synth.ar_series(n, p, rng, 0.3, 0.8)
    s, tau, order, _ = ctx.pacf_device(to_dev(y), pmax, 1e-10, estimator=c.EST_SKETCH,
                                       sketch=c.SKETCH_UNIFORM, gamma=gamma, seed=seed,
                                       request_id=rid)
    assert s == c.TLS_OK
    m = n - pmax
    rows = []
    for h in range(1, pmax + 1):
        ch = gamma * h
        u = oracle.philox_uniform(ch, c.RNG_UNIFORM_ROWS, rid + h - 1, seed)
        rows.append(oracle.uniform_rows(u, m, ch))
    ref = oracle.pacf_compressed(y, pmax, rows)
    err = np.abs(tau - ref).max()
    say("   max |tau - oracle| = %.3g, order %d" % (err, order))
    assert err <= 1e-10
    band_rows = [gamma * h for h in range(1, pmax + 1)]
    want = oracle.pacf_order(ref, band_rows)
    if np.all(np.abs(np.abs(ref) - 1.96 / np.sqrt(band_rows)) > 1e-6):
        assert order == want


def test_pacf_arguments(ctx):
    c = capi()
    y = to_dev(np.random.default_rng(0).standard_normal(3000))
    assert ctx.pacf_device(y, 0)[0] == c.TLS_EINVAL
    assert ctx.pacf_device(y, 1500)[0] == c.TLS_EINVAL  # n < 2 pmax + 1
    big = to_dev(np.random.default_rng(1).standard_normal(5000))
    assert ctx.pacf_device(big, 1025)[0] == c.TLS_EUNSUPPORTED
