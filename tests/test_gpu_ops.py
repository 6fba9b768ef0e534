"""Step-level parity: each HIP step, called through the C-ABI, against the FP64
CPU oracle on the same seeded inputs (element by element)."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import EPS32, EPS64, capi, fft_tol, say, to_dev, to_np, torch_dev, unpack_spectra

pytestmark = pytest.mark.gpu

# (n, p, B): several blocks with a ragged tail, p = 1, B = 2p, one large block,
# block length at both ends of the supported range.
CASES = [
    (200, 3, 128),
    (1000, 1, 128),
    (5000, 17, 256),
    (40000, 64, 128),
    (70000, 100, 2048),
    (3000, 500, 1024),
    (20000, 5, 16384),
    (100003, 200, 4096),
]


@pytest.fixture(scope="module")
def ctx():
    c = capi()
    with c.Context(0) as cx:
        yield cx


def _series(n, p, seed):
    rng = np.random.default_rng(seed)
    return synth.ar_series(n, min(p, 50), rng, 0.3, 0.9)


def _spec_dev(ctx, prec, y, p, B):
    c = capi()
    torch, dev = torch_dev()
    nb = c.num_blocks(y.size, p, B)
    dt = torch.float64 if prec == c.PREC_F64 else torch.float32
    spec = torch.zeros(nb * B, dtype=dt, device=dev)  # nb * B/2 complex words
    dy = to_dev(y)
    assert ctx.op_spectra(prec, dy, p, B, spec) == c.TLS_OK
    return spec, nb


def test_philox_matches_oracle(ctx):
    c = capi()
    torch, dev = torch_dev()
    say("philox")
    seed = (1 << 40) + 5
    out = torch.zeros(10000, dtype=torch.float64, device=dev)
    assert ctx.op_philox(seed, 3, 7, 123, 10000, out) == c.TLS_OK
    ref = oracle.philox_uniform(10000, 3, 7, seed, start=123)
    assert np.array_equal(to_np(out), ref)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,p,B", CASES)
def test_spectra(ctx, prec, n, p, B):
    say("spectra", prec, n, p, B)
    y = _series(n, p, 11)
    spec, nb = _spec_dev(ctx, prec, y, p, B)
    got = unpack_spectra(to_np(spec).astype(np.float64).view(np.complex128).reshape(nb, B // 2), B)
    ref = oracle.block_spectra(y, p, B)
    scale = np.abs(ref).max()
    tol = fft_tol(EPS64, B, scale) if prec == 0 else 2 * EPS32 * scale
    assert np.abs(got - ref).max() <= tol


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,p,B", CASES)
def test_toeplitz_mv(ctx, prec, n, p, B):
    """e = s1 X v + s2 w and ||e||^2 against dense products."""
    c = capi()
    torch, dev = torch_dev()
    say("toeplitz_mv", prec, n, p, B)
    rng = np.random.default_rng(5)
    y = _series(n, p, 12)
    m = n - p
    v = rng.standard_normal(p)
    w = rng.standard_normal(m)
    spec, nb = _spec_dev(ctx, prec, y, p, B)
    dt = torch.float64 if prec == 0 else torch.float32
    dw = to_dev(w, dt)
    de = torch.zeros(m, dtype=dt, device=dev)
    dout = torch.zeros(p + 1, dtype=torch.float64, device=dev)
    s1, s2 = -0.75, 1.25
    assert ctx.op_toeplitz(prec, spec, n, p, B, v=v, s1=s1, s2=s2, d_w=dw, d_e=de,
                           want_rmv=False, d_out=dout) == c.TLS_OK
    X, _ = oracle.lag_matrix(y, p)
    wr = w if prec == 0 else w.astype(np.float32).astype(np.float64)
    ref = s1 * (X @ v) + s2 * wr
    got = to_np(de).astype(np.float64)
    eps = EPS64 if prec == 0 else EPS32
    tol = fft_tol(eps, B, abs(s1) * np.abs(y).max() * np.abs(v).sum()) + 4 * eps * np.abs(ref).max()
    assert np.abs(got - ref).max() <= tol
    nrm = to_np(dout)[p]
    assert abs(nrm - ref @ ref) <= 1e-10 * (ref @ ref) if prec == 0 else abs(nrm - ref @ ref) <= 1e-4 * (ref @ ref)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,p,B", CASES)
def test_toeplitz_fused(ctx, prec, n, p, B):
    """One LSQR-shaped pass: e = s1 X v + s2 w stored in place of w, X^T e, ||e||^2."""
    c = capi()
    torch, dev = torch_dev()
    say("toeplitz_fused", prec, n, p, B)
    rng = np.random.default_rng(6)
    y = _series(n, p, 13)
    m = n - p
    v = rng.standard_normal(p)
    w = rng.standard_normal(m)
    spec, nb = _spec_dev(ctx, prec, y, p, B)
    dt = torch.float64 if prec == 0 else torch.float32
    dw = to_dev(w, dt)
    dout = torch.zeros(p + 1, dtype=torch.float64, device=dev)
    s1, s2 = 1.0, -0.3
    assert ctx.op_toeplitz(prec, spec, n, p, B, v=v, s1=s1, s2=s2, d_w=dw, d_e=dw,
                           want_rmv=True, d_out=dout) == c.TLS_OK
    X, _ = oracle.lag_matrix(y, p)
    wr = w if prec == 0 else w.astype(np.float32).astype(np.float64)
    e_ref = s1 * (X @ v) + s2 * wr
    e_got = to_np(dw).astype(np.float64)
    eps = EPS64 if prec == 0 else EPS32
    tol_e = fft_tol(eps, B, np.abs(y).max() * np.abs(v).sum()) + 4 * eps * np.abs(e_ref).max()
    assert np.abs(e_got - e_ref).max() <= tol_e
    g_ref = X.T @ e_got  # X^T of the vector the pass produced
    g = to_np(dout)[:p]
    tol_g = fft_tol(eps, B, np.abs(y).max() * np.abs(e_got).sum())
    assert np.abs(g - g_ref).max() <= tol_g


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,p,B", CASES[:6])
def test_toeplitz_rmv(ctx, prec, n, p, B):
    c = capi()
    torch, dev = torch_dev()
    say("toeplitz_rmv", prec, n, p, B)
    rng = np.random.default_rng(7)
    y = _series(n, p, 14)
    m = n - p
    u = rng.standard_normal(m)
    spec, nb = _spec_dev(ctx, prec, y, p, B)
    dt = torch.float64 if prec == 0 else torch.float32
    du = to_dev(u, dt)
    dout = torch.zeros(p + 1, dtype=torch.float64, device=dev)
    assert ctx.op_toeplitz(prec, spec, n, p, B, d_u_in=du, want_rmv=True, d_out=dout) == c.TLS_OK
    ur = u if prec == 0 else u.astype(np.float32).astype(np.float64)
    X, _ = oracle.lag_matrix(y, p)
    g_ref = X.T @ ur
    eps = EPS64 if prec == 0 else EPS32
    assert np.abs(to_np(dout)[:p] - g_ref).max() <= fft_tol(eps, B, np.abs(y).max() * np.abs(ur).sum())
    assert abs(to_np(dout)[p] - ur @ ur) <= 1e-12 * (ur @ ur)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,p,B,k", [(5000, 17, 256, 8), (70000, 100, 2048, 8), (3001, 4, 128, 3)])
def test_scores(ctx, prec, n, p, B, k):
    c = capi()
    torch, dev = torch_dev()
    say("scores", prec, n, p, B, k)
    rng = np.random.default_rng(8)
    y = _series(n, p, 15)
    Om = rng.standard_normal((p, k)) / np.sqrt(k)
    spec, nb = _spec_dev(ctx, prec, y, p, B)
    dt = torch.float64 if prec == 0 else torch.float32
    dom = to_dev(np.asfortranarray(Om).T.copy())  # columns contiguous
    ds = torch.zeros(n - p, dtype=dt, device=dev)
    assert ctx.op_scores(prec, spec, n, p, B, dom, k, ds) == c.TLS_OK
    ref = oracle.scores_from_omega(y, p, Om)
    got = to_np(ds).astype(np.float64)
    eps = EPS64 if prec == 0 else EPS32
    # each column product carries fft_tol; squares add 2x relative
    colmax = np.abs(y).max() * np.abs(Om).sum(axis=0).max()
    tol = 2 * k * colmax * fft_tol(eps, B, colmax) + 4 * eps * ref.max()
    assert np.abs(got - ref).max() <= tol


def test_sample_matches_oracle(ctx):
    c = capi()
    torch, dev = torch_dev()
    say("sample")
    rng = np.random.default_rng(9)
    m, cc = 50000, 777
    s = rng.uniform(0.0, 1.0, m) ** 3
    s[rng.choice(m, 500, replace=False)] = 0.0  # zero-score rows must never be drawn
    u = rng.random(cc)
    ds = to_dev(s)
    du = to_dev(u)
    idx = torch.zeros(cc, dtype=torch.int64, device=dev)
    sc = torch.zeros(cc, dtype=torch.float64, device=dev)
    assert ctx.op_sample(0, ds, m, du, cc, 0, 0, idx, sc) == c.TLS_OK
    ri, rs = oracle.leverage_sample(s, u, cc)
    gi, gs = to_np(idx), to_np(sc)
    total = s.sum()
    running = np.cumsum(s)
    mism = np.nonzero(gi != ri)[0]
    for t in mism:  # allowed only where the draw sits on a boundary within rounding
        assert abs(running[min(ri[t], gi[t])] - u[t] * total) <= 1e-12 * total, t
        assert s[gi[t]] > 0
    assert mism.size <= 2
    assert np.all(s[gi] > 0)
    ok = gi == ri
    assert np.allclose(gs[ok], rs[ok], rtol=1e-12)


def test_sample_philox_stream(ctx):
    """Without given draws the sampler uses Philox stream 3 of (seed, fit)."""
    c = capi()
    torch, dev = torch_dev()
    say("sample_philox")
    rng = np.random.default_rng(10)
    m, cc, seed, fit = 20000, 300, 99, 4
    s = rng.uniform(0.1, 1.0, m)
    idx = torch.zeros(cc, dtype=torch.int64, device=dev)
    sc = torch.zeros(cc, dtype=torch.float64, device=dev)
    assert ctx.op_sample(0, to_dev(s), m, None, cc, seed, fit, idx, sc) == c.TLS_OK
    u = oracle.philox_uniform(cc, c.RNG_LEVERAGE, fit, seed)
    ri, _ = oracle.leverage_sample(s, u, cc)
    gi = to_np(idx)
    total = s.sum()
    running = np.cumsum(s)
    mism = np.nonzero(gi != ri)[0]
    for t in mism:  # allowed only where the draw sits on a boundary within rounding
        assert abs(running[min(ri[t], gi[t])] - u[t] * total) <= 1e-12 * total, t
    assert mism.size <= 2


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_gather(ctx, mode):
    c = capi()
    torch, dev = torch_dev()
    say("gather", mode)
    rng = np.random.default_rng(11)
    n, p = 3000, 7
    m = n - p
    y = rng.standard_normal(n)
    ldq = 16
    if mode == 2:
        cc = m
    else:
        cc = 101
    crows = (cc + 15) // 16 * 16
    A = torch.full((crows * ldq,), 7.0, dtype=torch.float64, device=dev)
    seed, fit = 1234, 2
    if mode == 0:
        ri = rng.integers(0, m, cc)
        rs = rng.uniform(0.5, 2.0, cc)
        di, ds = to_dev(ri.astype(np.int64)), to_dev(rs)
    else:
        di = torch.zeros(cc, dtype=torch.int64, device=dev)
        ds = torch.zeros(cc, dtype=torch.float64, device=dev)
        if mode == 1:
            ri, rs = oracle.uniform_rows(oracle.philox_uniform(cc, c.RNG_UNIFORM_ROWS, fit, seed), m, cc)
        else:
            ri, rs = np.arange(m), np.ones(m)
    assert ctx.op_gather(to_dev(y), p, mode, di, ds, cc, crows, ldq, A, seed, fit) == c.TLS_OK
    got = to_np(A).reshape(crows, ldq)
    ref = oracle.sketch_rows(y, p, ri, rs)
    assert np.allclose(got[:cc, : p + 1], ref, rtol=1e-15, atol=0)
    assert np.all(got[:cc, p + 1:] == 0) and np.all(got[cc:] == 0)
    if mode == 1:
        assert np.array_equal(to_np(di), ri)


@pytest.mark.parametrize("c_rows,q,decades", [(64, 4, 3), (800, 101, 3), (2000, 65, 3), (400, 200, 3),
                                                (4000, 129, 3), (1792, 224, 3), (1808, 225, 3),
                                                (2400, 257, 3), (4008, 501, 3), (3000, 300, 7),
                                                (8200, 1025, 3), (800, 101, 12), (2400, 101, 13)])
def test_qr_matches_lapack(ctx, c_rows, q, decades):
    """Orders above 224 take the blocked Cholesky (32 x 32 blocks): whole and
    ragged last blocks, and columns scaled over 7 decades; at 12 and 13
    decades the unshifted sweeps can break down and are redone shifted."""
    c = capi()
    torch, dev = torch_dev()
    say("qr", c_rows, q, decades)
    rng = np.random.default_rng(12)
    ldq = (q + 15) // 16 * 16
    crows = (c_rows + 15) // 16 * 16
    A = np.zeros((crows, ldq))
    A[:c_rows, :q] = rng.standard_normal((c_rows, q)) @ np.diag(np.logspace(0, decades, q))
    dA = to_dev(A.ravel())
    dR = torch.zeros(q * q, dtype=torch.float64, device=dev)
    s, st = ctx.op_qr(dA, crows, q, ldq, dR)
    assert s == c.TLS_OK and st & 2 == 0
    R = to_np(dR).reshape(q, q)
    RL = oracle.qr_r(A[:c_rows, :q])
    RL = RL * np.sign(np.diag(RL))[:, None]
    assert np.all(np.diag(R) > 0)
    assert np.allclose(np.tril(R, -1), 0)
    k = oracle.kappa(RL)
    assert np.abs(R - RL).max() <= 1e-13 * k * np.abs(RL).max()
    G = A[:c_rows, :q].T @ A[:c_rows, :q]
    assert np.abs(R.T @ R - G).max() <= 1e-13 * np.abs(G).max() * q


def test_qr_flags_rank_deficiency(ctx):
    c = capi()
    torch, dev = torch_dev()
    say("qr_rank")
    rng = np.random.default_rng(13)
    A = np.zeros((64, 16))
    base = rng.standard_normal((64, 3))
    A[:, :3] = base
    A[:, 3] = base[:, 0] + base[:, 1]  # dependent column
    dR = torch.zeros(16, dtype=torch.float64, device=dev)
    s, st = ctx.op_qr(to_dev(A.ravel()), 64, 4, 16, dR)
    assert s == c.TLS_OK and (st & 6)


@pytest.mark.parametrize("p", [1, 3, 37, 100, 128, 129, 150, 224, 225, 256, 300, 500, 1024])
def test_triinv(ctx, p):
    c = capi()
    torch, dev = torch_dev()
    say("triinv", p)
    rng = np.random.default_rng(14)
    q = p + 1
    R = np.triu(rng.standard_normal((q, q))) + np.diag(2 + rng.random(q))
    dM = torch.zeros(p * p, dtype=torch.float64, device=dev)
    dphi = torch.zeros(p, dtype=torch.float64, device=dev)
    assert ctx.op_triinv(to_dev(R.ravel()), q, p, dM, dphi) == c.TLS_OK
    Mref = oracle.tri_inverse(R[:p, :p])
    M = to_np(dM).reshape(p, p)
    k = oracle.kappa(R[:p, :p])
    assert np.abs(M - Mref).max() <= 1e-14 * k * np.abs(Mref).max() * p
    assert np.allclose(to_np(dphi), Mref @ R[:p, p], rtol=1e-10, atol=1e-12 * np.abs(Mref @ R[:p, p]).max())


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("p,k,extra", [(5, 8, 1), (100, 8, 1), (37, 3, 4), (64, 8, 0),
                                       (200, 8, 1), (300, 5, 3), (700, 8, 1)])
def test_jl_map(ctx, kind, p, k, extra):
    """Pi from the Philox streams, and Omega = R[:p,:p]^{-1} Pi^T by back
    substitution against a LAPACK triangular solve; R has q = p + extra
    columns and NaN below its diagonal, which must not be read."""
    c = capi()
    torch, dev = torch_dev()
    say("jl", kind, p, k, extra)
    rng = np.random.default_rng(15 + p)
    q = p + extra
    R = np.triu(rng.standard_normal((q, q))) / np.sqrt(q) + 3 * np.eye(q)
    R[np.tril_indices(q, -1)] = np.nan
    seed, fit = 77, 5
    dPi = torch.zeros(k * p, dtype=torch.float64, device=dev)
    dOm = torch.zeros(k * p, dtype=torch.float64, device=dev)
    assert ctx.op_jl(to_dev(R.ravel()), q, p, k, kind, seed, fit, dPi, dOm) == c.TLS_OK
    Pi = to_np(dPi).reshape(k, p)
    P = 1 << max(0, math.ceil(math.log2(p)))
    if kind == 0:
        ref = oracle.srht_map(p, k, oracle.philox_uniform(P, c.RNG_SRHT_SIGNS, fit, seed),
                              oracle.philox_uniform(k, c.RNG_SRHT_ROWS, fit, seed))
        assert np.allclose(Pi, ref, rtol=1e-15, atol=0)
    else:
        ref = oracle.philox_normal(k * p, c.RNG_GAUSS, fit, seed).reshape(k, p) / np.sqrt(k)
        assert np.allclose(Pi, ref, rtol=1e-13, atol=1e-15)
    Ru = np.triu(np.nan_to_num(R[:p, :p]))
    want = oracle.jl_omega(Ru, Pi)
    Om = to_np(dOm).reshape(k, p).T
    kap = oracle.kappa(Ru)
    assert np.isfinite(Om).all()
    assert np.abs(Om - want).max() <= 4 * p * 2.0 ** -53 * kap * np.abs(want).max()
