"""The allocation-free pass (tls_op_toeplitz_noalloc) against tls_op_toeplitz.

Both run the same kernels on the same inputs, so outputs must agree bit for
bit; the no-allocation call keeps its scratch in a fixed per-device array that
keeps the previous call's contents, so two calls in a row (the second on a
smaller problem) are checked, and the result is also checked against the
oracle's dense products."""
import numpy as np
import pytest

import oracle
from gpu_common import EPS32, EPS64, capi, fft_tol, say, to_dev, to_np, torch_dev

pytestmark = pytest.mark.gpu


def _series(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


def _spec(ctx, prec, y, p, B):
    torch, dev = torch_dev()
    c = capi()
    nb = c.lib.tls_num_blocks(y.size, p, B)
    words = nb * (B // 2) * (2 if prec == 0 else 1)
    spec = torch.zeros(words, dtype=torch.float64, device=dev)
    assert ctx.op_spectra(prec, to_dev(y), p, B, spec) == c.TLS_OK
    return spec


def _run(ctx, fn, prec, spec, y, p, B, v, w):
    torch, dev = torch_dev()
    dt = torch.float64 if prec == 0 else torch.float32
    dw = to_dev(w, dt)
    dout = torch.zeros(p + 1, dtype=torch.float64, device=dev)
    st = fn(prec, spec, y.size, p, B, v=v, s1=0.8, s2=-0.45, d_w=dw, d_e=dw, want_rmv=True,
            d_out=dout)
    assert st == capi().TLS_OK, st
    return to_np(dw), to_np(dout)


# (n, p, B, prec): several blocks and a ragged last block each; the second of
# each pair is smaller than the first
PAIRS = [((60001, 37, 256, 0), (9001, 12, 128, 0)),
         ((200003, 100, 1024, 0), (30011, 3, 512, 0)),
         ((150007, 64, 2048, 1), (20011, 9, 256, 1))]


@pytest.mark.parametrize("first,second", PAIRS)
def test_noalloc_matches_workspace_pass(first, second):
    c = capi()
    with c.Context(0) as ctx:
        for k, (n, p, B, prec) in enumerate((first, second)):
            say("noalloc", k, n, p, B, prec)
            y = _series(n, 100 + n % 97)
            rng = np.random.default_rng(n)
            v = rng.standard_normal(p)
            w = rng.standard_normal(n - p)
            spec = _spec(ctx, prec, y, p, B)
            e_ws, out_ws = _run(ctx, ctx.op_toeplitz, prec, spec, y, p, B, v, w)
            e_na, out_na = _run(ctx, ctx.op_toeplitz_noalloc, prec, spec, y, p, B, v, w)
            assert np.array_equal(e_na, e_ws)
            assert np.array_equal(out_na, out_ws)
            # and the products themselves against the oracle's dense ones
            X, _ = oracle.lag_matrix(y, p)
            wr = w if prec == 0 else w.astype(np.float32).astype(np.float64)
            e_ref = 0.8 * (X @ v) - 0.45 * wr
            eps = EPS64 if prec == 0 else EPS32
            e64 = e_na.astype(np.float64)
            tol_e = fft_tol(eps, B, np.abs(y).max() * np.abs(v).sum()) + 4 * eps * np.abs(e_ref).max()
            assert np.abs(e64 - e_ref).max() <= tol_e
            tol_g = fft_tol(eps, B, np.abs(y).max() * np.abs(e64).sum())
            assert np.abs(out_na[:p] - X.T @ e64).max() <= tol_g
            assert abs(out_na[p] - e64 @ e64) <= (1e-12 if prec == 0 else 1e-5) * (e64 @ e64)


def test_noalloc_rejects_oversized_scratch():
    """p = 1000, B = 2048: 4194 blocks in 2097 groups need 1001 x 2097 partial
    sums (16.8 MB) beyond the 16 MiB array; rejected before any work."""
    c = capi()
    torch, dev = torch_dev()
    n, p, B = 4_400_000, 1000, 2048
    nb = c.lib.tls_num_blocks(n, p, B)
    assert nb == 4194
    with c.Context(0) as ctx:
        spec = torch.zeros(nb * (B // 2) * 2, dtype=torch.float64, device=dev)
        u = torch.zeros(n - p, dtype=torch.float64, device=dev)
        out = torch.zeros(p + 1, dtype=torch.float64, device=dev)
        st = ctx.op_toeplitz_noalloc(0, spec, n, p, B, v=np.ones(p), d_w=u, d_e=u, d_out=out)
        assert st == c.TLS_EUNSUPPORTED
        assert ctx.op_toeplitz(0, spec, n, p, B, v=np.ones(p), d_w=u, d_e=u, d_out=out) == c.TLS_OK
