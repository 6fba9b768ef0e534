"""Parity on the configured workloads against the FP64 QR oracle.

- AR(100), n = 2^22, seeds 1..9 (the kappa-stratified sweep beside seed 0),
  FP64 at the configured 8p sketch, against the stored oracle solutions
  (tests/golden/make_config_oracles.py).
- AR(500): the first 2^20 samples of the seed-0 series, FP64 and mixed
  precision, on the full-size plan's block length B = 4096.
- Served requests (continuous batching) against the oracle itself.
- The default-context call tls_fit on the AR(3) workload.

Gates: 1e-6 (FP64) and 1e-4 (mixed) on the coefficients wherever the
attainable accuracy (gpu_common.attainable) is below them; fitted values and
the residual norm against their derived bounds at any conditioning."""
import os

import numpy as np
import pytest

import oracle
import synth
from tests.conftest import GOLDEN
from tests.gpu_common import attainable, capi, chunked_matvec_norms, resid_tol, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = capi()
    with c.Context(0) as cx:
        yield cx


def _stored(name):
    data = np.loadtxt(os.path.join(GOLDEN, name))
    return data[:-3], data[-3], data[-2], data[-1]  # phi, ||r*||, kappa, ||X||


def _check_against(out, y, p, phi, rnorm, kappa, smax, gate, tol=1e-10, what=""):
    c = capi()
    xd, xphi = chunked_matvec_norms(y, p, out["coef"] - phi, phi)
    coef_b, fit_b = attainable(phi, rnorm, kappa, smax, xphi, float(np.linalg.norm(y[p:])), p,
                               out["block_len"], tol)
    err = oracle.rel_error(out["coef"], phi)
    say("   %s kappa=%.3g err=%.3g (bound %.2g) fit=%.3g (bound %.2g) iters=%d status=%s"
        % (what, kappa, err, coef_b, xd / xphi, fit_b, out["iters"],
           c.status_string(out["status"])))
    if out["status"] == c.TLS_ESTALL:
        assert out["istop"] == 5 and coef_b > gate, (coef_b, out["istop"])
    else:
        assert out["status"] == c.TLS_OK, c.status_string(out["status"])
    if coef_b < gate:
        assert err <= gate
    assert xd / xphi <= max(10 * fit_b, 1e-14)
    assert abs(out["resid_norm"] - rnorm) <= resid_tol(phi, rnorm, smax, np.abs(y).max(), p, xd)
    return err, coef_b


@pytest.mark.parametrize("seed", range(1, 10))
def test_ar100_seeds_against_stored_oracle(ctx, seed):
    say("ar100 seed", seed)
    phi, rnorm, kappa, smax = _stored(f"ar100_seed{seed}_oracle.txt")
    f = synth.workload_ar100(seed=seed)
    assert f.gamma == 8 and f.y.size == 1 << 22
    out = ctx.fit_device(to_dev(f.y), 100, f.tol, gamma=f.gamma)
    _check_against(out, f.y, 100, phi, rnorm, kappa, smax, 1e-6, f.tol, "f64")


@pytest.mark.parametrize("precision", [0, 1])
def test_ar500_prefix_against_stored_oracle(ctx, precision):
    """The configured AR(500) generator (pole moduli U[0.5, 0.95]) on the
    2^20-sample prefix the oracle can factor; B = 4096 as at full size."""
    say("ar500 prefix", precision)
    phi, rnorm, kappa, smax = _stored("ar500_prefix_oracle.txt")
    y = synth.workload_ar500(seed=0).y[: 1 << 20]
    out = ctx.fit_device(to_dev(y), 500, 1e-10, precision=precision, block_lg=12)
    assert out["block_len"] == 4096
    _check_against(out, y, 500, phi, rnorm, kappa, smax, 1e-6 if precision == 0 else 1e-4,
                   1e-10, "mixed" if precision else "f64")


def test_served_requests_against_oracle(ctx):
    """Requests in flight together (varied n and p) each against the oracle."""
    c = capi()
    say("serve vs oracle")
    rng = np.random.default_rng(77)
    work = []
    for _ in range(12):
        p = int(rng.integers(2, 80))
        n = int(round(2.0 ** rng.uniform(11, 16)))
        work.append((synth.ar_series(n, p, rng, 0.5, 0.95), p))
    with c.Server(ctx, 1 << 30, 64) as srv:
        tickets = [srv.submit_device(to_dev(y), p, 1e-10, request_id=500 + i)
                   for i, (y, p) in enumerate(work)]
        outs = [srv.wait(t) for t in tickets]
    for (y, p), o in zip(work, outs):
        ref = oracle.fit_qr(y, p)
        smax = float(np.linalg.svd(ref["R"], compute_uv=False)[0])
        _check_against(o, y, p, ref["phi"], ref["rnorm"], ref["kappa"], smax, 1e-6,
                       what=f"served p={p} n={y.size}")


def test_default_context_tls_fit(ctx):
    """tls_fit (default context: device 0, default options) on the AR(3)
    workload against the oracle."""
    c = capi()
    say("tls_fit default context")
    f = synth.workload_ar3(seed=0)
    s, coef, rn, iters = c.tls_fit(f.y, 3, 1e-10)
    assert s == c.TLS_OK and iters >= 1
    ref = oracle.fit_qr(f.y, 3)
    assert oracle.rel_error(coef, ref["phi"]) <= 1e-9
    assert abs(rn - ref["rnorm"]) <= 1e-9 * ref["rnorm"]
    # a second call reuses the default context and gives the same result
    s2, coef2, rn2, _ = c.tls_fit(f.y, 3, 1e-10)
    assert s2 == c.TLS_OK and coef2.tobytes() == coef.tobytes() and rn2 == rn
