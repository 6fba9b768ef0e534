"""Served continuous batching (tls_server_*): every request's result equals the
single fit with the same options and request id bit for bit, whatever else is
in flight; admission under a small HBM budget; concurrent submitters;
rejected submissions; rank-deficient and degenerate requests; mixed
precision, where each request takes its own path (FP32-product or FP64 LSQR)
inside the same tick."""
import threading

import numpy as np
import pytest

import synth
from tests.gpu_common import capi, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = capi()
    with c.Context(0) as cx:
        yield cx


def _series(seed, count, lo=10, hi=16, pmax=120):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        p = int(rng.integers(2, pmax + 1))
        n = int(round(2.0 ** rng.uniform(lo, hi)))
        n = max(n, 2 * p + 1)
        out.append((synth.ar_series(n, p, rng, 0.3, 0.9), p))
    return out


def _check_same(ctx, y, p, rid, got, **opts):
    single = ctx.fit_device(to_dev(y), p, 1e-10, request_id=rid, **opts)
    assert got["status"] == single["status"], (rid, p, y.size)
    assert got["coef"].tobytes() == single["coef"].tobytes(), (rid, p, y.size)
    assert got["iters"] == single["iters"], (rid, p, y.size)
    assert got["resid_norm"] == single["resid_norm"], (rid, p, y.size)
    assert got["mixed_path"] == single["mixed_path"], (rid, p, y.size)


def test_serve_device_equals_single(ctx):
    c = capi()
    say("serve device")
    work = _series(1, 40)
    with c.Server(ctx, 2 << 30, 64) as srv:
        devs = [to_dev(y) for y, _ in work]
        tickets = [srv.submit_device(d, p, 1e-10, request_id=1000 + i)
                   for i, (d, (_, p)) in enumerate(zip(devs, work))]
        outs = [srv.wait(t) for t in tickets]
        st = srv.stats()
    say("   ticks", st["ticks"], "completed", st["completed"])
    assert st["completed"] == len(work) and st["in_flight"] == 0 and st["queued"] == 0
    for i, ((y, p), o) in enumerate(zip(work, outs)):
        _check_same(ctx, y, p, 1000 + i, o)
        assert o["t_total_ms"] > 0


def test_serve_host_small_budget_queues(ctx):
    """A budget that holds only a few fits at once: requests wait for
    admission in order and all finish with their single-fit results."""
    c = capi()
    say("serve host small budget")
    work = _series(2, 12, lo=12, hi=14, pmax=30)
    with c.Server(ctx, 2 << 20, 16) as srv:
        tickets = [srv.submit(y, p, 1e-10, request_id=i) for i, (y, p) in enumerate(work)]
        outs = [srv.wait(t) for t in tickets]
        st = srv.stats()
    say("   ticks", st["ticks"])
    assert st["completed"] == len(work)
    for i, ((y, p), o) in enumerate(zip(work, outs)):
        _check_same(ctx, y, p, i, o)


def test_serve_concurrent_submitters(ctx):
    c = capi()
    say("serve concurrent")
    work = _series(3, 24, lo=10, hi=15)
    devs = [to_dev(y) for y, _ in work]
    tickets = [None] * len(work)
    with c.Server(ctx, 1 << 30, 32) as srv:
        def submitter(part):
            for i in part:
                tickets[i] = srv.submit_device(devs[i], work[i][1], 1e-10, request_id=50 + i)

        th = [threading.Thread(target=submitter, args=(range(k, len(work), 3),)) for k in range(3)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        outs = {}
        while len(outs) < len(work):
            for i, t in enumerate(tickets):
                if i not in outs:
                    r = srv.poll(t)
                    if r is not None:
                        outs[i] = r
    for i, (y, p) in enumerate(work):
        _check_same(ctx, y, p, 50 + i, outs[i])


def test_serve_rejections(ctx):
    c = capi()
    say("serve rejections")
    rng = np.random.default_rng(4)
    y = synth.ar_series(5000, 5, rng, 0.3, 0.9)
    with c.Server(ctx, 4 << 20, 4) as srv:
        with pytest.raises(c.TlsError) as e:
            srv.submit(y, 0, 1e-10)
        assert e.value.status == c.TLS_EINVAL
        bad = y.copy()
        bad[3] = np.nan
        with pytest.raises(c.TlsError) as e:
            srv.submit(bad, 5, 1e-10)
        assert e.value.status == c.TLS_EINVAL
        with pytest.raises(c.TlsError) as e:
            srv.submit(y, 624, 1e-10)  # above the batched kernels' largest order, 623
        assert e.value.status == c.TLS_EUNSUPPORTED
        big = synth.ar_series(1 << 18, 5, rng, 0.3, 0.9)
        with pytest.raises(c.TlsError) as e:
            srv.submit(big, 5, 1e-10)  # footprint above the 4 MiB budget
        assert e.value.status == c.TLS_ENOMEM
        with pytest.raises(c.TlsError) as e:
            srv.wait(123456789)
        assert e.value.status == c.TLS_EINVAL
        t = srv.submit(y, 5, 1e-10)
        assert srv.wait(t)["status"] == c.TLS_OK
    with pytest.raises(c.TlsError) as e:
        c.Server(ctx, 1 << 30, 8, precision=1, max_refine=4)  # no refinement when served
    assert e.value.status == c.TLS_EUNSUPPORTED
    with pytest.raises(c.TlsError) as e:
        c.Server(ctx, 1 << 30, 8, precision=2)
    assert e.value.status == c.TLS_EINVAL


def test_serve_degenerate_requests(ctx):
    """Rank-one (constant) series, minimal length, all-rows sketch, mixed in
    with ordinary requests."""
    c = capi()
    say("serve degenerate")
    rng = np.random.default_rng(5)
    reqs = [(np.full(3000, 2.0), 3), (rng.standard_normal(13), 6),
            (synth.ar_series(300, 20, rng, 0.3, 0.9), 20), (synth.ar_series(20000, 8, rng, 0.3, 0.9), 8)]
    with c.Server(ctx, 256 << 20, 8) as srv:
        tickets = [srv.submit(y, p, 1e-10, request_id=70 + i) for i, (y, p) in enumerate(reqs)]
        outs = [srv.wait(t) for t in tickets]
    assert outs[0]["status"] == c.TLS_ERANK
    for i, ((y, p), o) in enumerate(zip(reqs, outs)):
        single = ctx.fit(y, p, 1e-10, request_id=70 + i)
        assert o["status"] == single["status"]
        assert o["coef"].tobytes() == single["coef"].tobytes()


def test_serve_destroy_with_requests_in_flight(ctx):
    c = capi()
    say("serve destroy in flight")
    work = _series(6, 10, lo=12, hi=16)
    srv = c.Server(ctx, 512 << 20, 8)
    for i, (y, p) in enumerate(work):
        srv.submit(y, p, 1e-10, request_id=i)
    srv.close()  # runs everything to completion, discards the results


@pytest.mark.parametrize("tick_steps", [1, 7])
def test_serve_tick_steps_equal_single(ctx, tick_steps):
    """Any number of LSQR steps per tick gives every request its single-fit
    result (fits that converge inside a tick skip its remaining steps)."""
    c = capi()
    say("serve tick steps", tick_steps)
    work = _series(7, 16, lo=10, hi=15)
    with c.Server(ctx, 1 << 30, 32, tick_steps=tick_steps) as srv:
        tickets = [srv.submit_device(to_dev(y), p, 1e-10, request_id=300 + i)
                   for i, (y, p) in enumerate(work)]
        outs = [srv.wait(t) for t in tickets]
    for i, ((y, p), o) in enumerate(zip(work, outs)):
        _check_same(ctx, y, p, 300 + i, o)


@pytest.mark.parametrize("tick_steps", [1, 5])
def test_serve_mixed_equals_single(ctx, tick_steps):
    """A mixed-precision server: well and badly conditioned requests in flight
    together, each on the path its kappa_F selects, equal the single mixed fit
    bit for bit."""
    c = capi()
    say("serve mixed", tick_steps)
    rng = np.random.default_rng(8)
    work = []
    for i in range(24):
        p = int(rng.integers(2, 100))
        n = max(int(round(2.0 ** rng.uniform(11, 16))), 2 * p + 1)
        lo, hi = (0.3, 0.6) if i % 2 else (0.5, 0.95)
        work.append((synth.ar_series(n, p, rng, lo, hi), p))
    with c.Server(ctx, 1 << 30, 32, tick_steps=tick_steps, precision=1) as srv:
        tickets = [srv.submit_device(to_dev(y), p, 1e-10, request_id=700 + i)
                   for i, (y, p) in enumerate(work)]
        outs = [srv.wait(t) for t in tickets]
    paths = [o["mixed_path"] for o in outs]
    say("   paths", paths)
    assert 1 in paths and 3 in paths and 2 not in paths
    for i, ((y, p), o) in enumerate(zip(work, outs)):
        _check_same(ctx, y, p, 700 + i, o, precision=1)
