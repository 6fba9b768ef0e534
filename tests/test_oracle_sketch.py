"""Pins for oracle.sketch and oracle.philox: hand-worked sampling example,
unbiasedness of the rescaled sampling matrix, Definition 2.4 written out,
SRHT norm preservation in expectation, and the published Philox vectors."""
import numpy as np
import pytest

import oracle
import synth
from tests.conftest import read_golden


def test_inverse_cdf_hand_example():
    scores_s, rows = read_golden("inverse_cdf_example.txt")
    scores = np.array(scores_s[0], float)
    u = np.array([float(r[0]) for r in rows])
    expect = np.array([int(r[1]) for r in rows])
    idx, scale = oracle.leverage_sample(scores, u)
    assert np.array_equal(idx, expect)
    pi = scores[expect] / scores.sum()
    assert np.allclose(scale, 1.0 / np.sqrt(u.size * pi))


def test_uniform_rows_alg1():
    idx, scale = oracle.uniform_rows([0.0, 0.5, 0.999999], 10, c=3)
    assert list(idx) == [0, 5, 9]
    assert np.allclose(scale, np.sqrt(10 / 3))


def test_sampling_matrix_unbiased(rng):
    """E[S^T S] = I for leverage-score sampling with 1/sqrt(c pi) rescaling
    (Section 2.1.2): so E[(SA)^T (SA)] = A^T A.  Monte Carlo, 5 sigma."""
    scores = rng.uniform(0.1, 2.0, 12)
    c, trials = 20, 20000
    diag = np.zeros(12)
    for _ in range(trials):
        idx, scale = oracle.leverage_sample(scores, rng.random(c))
        np.add.at(diag, idx, scale ** 2)
    est = diag / trials
    pi = scores / scores.sum()
    sd = np.sqrt((1 - pi) / (c * pi) / trials)
    assert np.all(np.abs(est - 1.0) <= 5 * sd)


def test_sketch_rows_rescale(rng):
    y = rng.standard_normal(50)
    X, b = oracle.lag_matrix(y, 4)
    idx = np.array([3, 0, 45, 3])
    sc = np.array([1.0, 2.0, 0.5, -1.0])
    S = oracle.sketch_rows(y, 4, idx, sc)
    for t in range(4):
        assert np.array_equal(S[t, :4], X[idx[t]] * sc[t])
        assert S[t, 4] == b[idx[t]] * sc[t]


def test_hadamard_definition():
    H2 = np.array(read_golden("hadamard_h2.txt")[0], float) / 2.0
    assert np.allclose(oracle.hadamard(2), H2, atol=0)
    assert np.allclose(oracle.hadamard(1), np.array([[1, 1], [1, -1]]) / np.sqrt(2))
    for m in range(0, 7):
        H = oracle.hadamard(m)
        assert np.allclose(H.T @ H, np.eye(2 ** m), atol=1e-13)


def test_srht_map_preserves_norm_in_expectation(rng):
    p, k = 11, 4
    x = rng.standard_normal(p)
    acc, trials = 0.0, 20000
    vals = []
    for _ in range(trials):
        Pi = oracle.srht_map(p, k, rng.random(16), rng.random(k))
        vals.append(np.sum((Pi @ x) ** 2))
    vals = np.array(vals)
    assert abs(vals.mean() - x @ x) <= 5 * vals.std() / np.sqrt(trials)


def test_srht_columns_exact():
    """With all signs + and k = P rows picking each row once, the map is
    sqrt(P/k) H = H restricted to the first p columns."""
    p, P = 3, 4
    u_rows = (np.arange(P) + 0.5) / P
    Pi = oracle.srht_map(p, P, np.zeros(P), u_rows)
    assert np.allclose(Pi, oracle.hadamard(2)[:, :p])


def test_philox_known_answers():
    for row in read_golden("philox4x32_10_kat.txt")[0]:
        vals = [int(x, 16) for x in row]
        assert oracle.philox4x32_10(vals[0:4], vals[4:6]) == tuple(vals[6:10])


def test_philox_uniform_stream_layout():
    """philox_uniform draw j equals the scalar block at counter (j,0,s,f)."""
    seed, s, f = 0x1234_5678_9ABC, 3, 17
    u = oracle.philox_uniform(5, s, f, seed, start=7)
    for t in range(5):
        x0, x1, _, _ = oracle.philox4x32_10((7 + t, 0, s, f), (seed & 0xFFFFFFFF, seed >> 32))
        bits = ((x0 << 32) | x1) >> 12
        assert u[t] == (bits + 0.5) * 2.0 ** -52
    assert np.all((u > 0) & (u < 1))


def test_philox_uniform_moments():
    u = oracle.philox_uniform(200000, 1, 0, 42)
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / u.size)
    z = oracle.philox_normal(100000, 2, 0, 42)
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)


def test_compressed_solution_all_rows_is_ols(rng):
    """With every row at unit scale the compressed problem is the full one."""
    y = synth.ar_series(600, 5, rng, 0.3, 0.9)
    m = y.size - 5
    A = oracle.sketch_rows(y, 5, np.arange(m), np.ones(m))
    ref = oracle.fit_qr(y, 5)["phi"]
    assert oracle.rel_error(oracle.compressed_solution(A), ref) <= 1e-12


def test_compressed_solution_noise_free_recovery(rng):
    """A noise-free AR(3) recursion is solved exactly by any p or more
    independent sampled rows, whatever their scales."""
    phi = np.array([0.5, -0.3, 0.1])
    y = np.zeros(400)
    y[:3] = [1.0, -0.7, 0.4]
    for t in range(3, y.size):
        y[t] = phi[0] * y[t - 1] + phi[1] * y[t - 2] + phi[2] * y[t - 3]
    m = y.size - 3
    idx = rng.integers(0, 60, 12)  # early rows, before the recursion decays
    A = oracle.sketch_rows(y, 3, idx, rng.uniform(0.5, 3.0, idx.size))
    assert oracle.rel_error(oracle.compressed_solution(A), phi) <= 1e-10


def test_compressed_solution_p1_closed_form(rng):
    """p = 1: phi = sum s^2 x b / sum s^2 x^2 over the sampled rows."""
    y = rng.standard_normal(300)
    idx = rng.integers(0, 299, 40)
    s = rng.uniform(0.2, 2.0, 40)
    x, b = y[idx], y[idx + 1]
    want = np.sum(s * s * x * b) / np.sum(s * s * x * x)
    got = oracle.compressed_solution(oracle.sketch_rows(y, 1, idx, s))[0]
    assert abs(got - want) <= 1e-13 * abs(want)


def test_compressed_solution_scale_and_duplication_invariant(rng):
    y = synth.ar_series(800, 6, rng, 0.3, 0.9)
    idx = rng.integers(0, 794, 50)
    A = oracle.sketch_rows(y, 6, idx, np.ones(50))
    a = oracle.compressed_solution(A)
    assert oracle.rel_error(oracle.compressed_solution(3.7 * A), a) <= 1e-13
    assert oracle.rel_error(oracle.compressed_solution(np.vstack([A, A])), a) <= 1e-13


def test_rh_levels_are_nested_halvings():
    """Algorithm 4's halvings: each level is contained in the one below and
    holds about half its rows; the level count stops at <= c rows."""
    m = 1 << 16
    u = oracle.philox_uniform(m, 5, 3, 11)
    prev = np.ones(m, dtype=bool)
    for lev in range(1, 8):
        cur = oracle.rh_level_mask(u, lev)
        assert np.all(prev[cur])  # nested
        frac = cur.sum() / max(prev.sum(), 1)
        assert abs(frac - 0.5) <= 4 * np.sqrt(0.25 / prev.sum())
        prev = cur
    assert oracle.rh_levels(4194204, 800) == 13  # 4194204 / 2^13 = 512 <= 800 < 1024
    assert oracle.rh_levels(1000, 800) == 1
    assert oracle.rh_levels(1601, 800) == 1  # one halving leaves 800 rows
    assert oracle.rh_levels(1602, 800) == 2


def test_philox_normal_box_muller_hand_values():
    """Two normals worked by hand from the published Philox vector and the
    Box-Muller pairing (golden/philox_normal_box_muller.txt): a swap of cos
    and sin, or of the pair's order, or another pairing stride fails."""
    (rows,) = read_golden("philox_normal_box_muller.txt")
    want = np.array([float(r[1]) for r in rows])
    got = oracle.philox_normal(want.size, 0, 0, 0)
    np.testing.assert_allclose(got, want, rtol=2e-15, atol=0)
    # its uniforms are the KAT-derived draws the fixture lists
    u = oracle.philox_uniform(4, 0, 0, 0)
    assert u[0] == (1797145537418908 + 0.5) * 2.0 ** -52
    assert u[2] == (87592411667571 + 0.5) * 2.0 ** -52


def test_rh_sketch_one_level_is_the_leverage_sketch(rng):
    """Algorithm 4 with one level (c >= m / 2): uniform trials, eq. (glev)
    scores w.r.t. them, leverage sampling, built here step by step from the
    oracle's pinned parts."""
    y = synth.ar_series(1200, 4, rng, 0.3, 0.9)
    p, k = 4, 6
    m = y.size - p
    c = m // 2 + 5
    assert oracle.rh_levels(m, c) == 1
    uu, ul = rng.random(c), rng.random(m)
    Pi = rng.standard_normal((k, p)) / np.sqrt(k)
    d0 = rng.random(c)
    A, idx, scale, levels = oracle.rh_sketch(y, p, c, uu, ul, Pi, [d0])
    assert levels == 1
    i0, s0 = oracle.uniform_rows(uu, m, c)
    B = oracle.sketch_rows(y, p, i0, s0)
    R = oracle.shifted_r(B, p)
    sc = oracle.scores_from_omega(y, p, oracle.jl_omega(R, Pi))
    i1, s1 = oracle.leverage_sample(sc, d0, c)
    assert np.array_equal(idx, i1)
    np.testing.assert_allclose(scale, s1, rtol=1e-10)
    np.testing.assert_allclose(A, oracle.sketch_rows(y, p, i1, s1), rtol=1e-10)


def test_rh_sketch_levels_and_exact_scores(rng):
    """Several levels: the top level (0) draws from all rows, rows drawn at a
    level above 0 lie in that level (checked through the scores by rerunning
    the level step); with k = p and Pi = I the top-level scores are the exact
    generalised scores (Definition 3.6) w.r.t. the level-1 sketch."""
    y = synth.ar_series(6000, 3, rng, 0.3, 0.9)
    p = 3
    m = y.size - p
    c = 400
    levels = oracle.rh_levels(m, c)
    assert levels >= 3
    uu, ul = rng.random(c), rng.random(m)
    draws = [rng.random(c) for _ in range(levels)]
    Pi = np.eye(p)
    A, idx, scale, lv = oracle.rh_sketch(y, p, c, uu, ul, Pi, draws)
    assert lv == levels
    # level 0 reaches rows outside level 1 (about half of the draws)
    outside = ~oracle.rh_level_mask(ul, 1)[idx]
    assert 0.3 < outside.mean() < 0.7
    # rebuild the chain by hand to check level membership at every level
    i, s = oracle.uniform_rows(uu, m, c)
    B = oracle.sketch_rows(y, p, i, s)
    X, _ = oracle.lag_matrix(y, p)
    for lev in range(levels - 1, -1, -1):
        R = oracle.shifted_r(B, p)
        sc = oracle.scores_from_omega(y, p, oracle.jl_omega(R, Pi))
        if lev == 0:
            np.testing.assert_allclose(sc, oracle.generalized_scores(X, B[:, :p]), rtol=1e-9)
        else:
            sc = np.where(oracle.rh_level_mask(ul, lev), sc, 0.0)
        i, s = oracle.leverage_sample(sc, draws[lev], c)
        if lev > 0:
            assert np.all(oracle.rh_level_mask(ul, lev)[i])
        B = oracle.sketch_rows(y, p, i, s)
    assert np.array_equal(i, idx)
    np.testing.assert_allclose(B, A, rtol=1e-12)


def test_sketch_r_sign_convention(rng):
    """sketch_r: upper triangular, non-negative diagonal, R^T R = A^T A, and
    equal to the transposed Cholesky factor of A^T A (the factor that a
    Cholesky-based QR produces), whatever signs the Householder QR chose."""
    A = rng.standard_normal((40, 6)) * np.array([1, 10, 0.1, 3, 1e3, 1])
    R = oracle.sketch_r(A, 5)
    assert np.all(np.diag(R) >= 0) and np.allclose(R, np.triu(R))
    np.testing.assert_allclose(R.T @ R, A[:, :5].T @ A[:, :5], rtol=1e-12, atol=1e-9)
    L = np.linalg.cholesky(A[:, :5].T @ A[:, :5])
    np.testing.assert_allclose(R, L.T, rtol=1e-9, atol=1e-9 * np.abs(L).max())
    # flipping a row of A's QR factor changes the JL scores but not the exact ones
    Pi = rng.standard_normal((3, 5))
    D = np.diag([1, -1, 1, 1, -1.0])
    y = synth.ar_series(400, 5, rng, 0.3, 0.8)
    a = oracle.scores_from_omega(y, 5, oracle.jl_omega(R, Pi))
    b = oracle.scores_from_omega(y, 5, oracle.jl_omega(D @ R, Pi))
    assert np.abs(a - b).max() > 1e-6 * np.abs(a).max()
    e1 = oracle.scores_from_omega(y, 5, oracle.jl_omega(R, np.eye(5)))
    e2 = oracle.scores_from_omega(y, 5, oracle.jl_omega(D @ R, np.eye(5)))
    np.testing.assert_allclose(e1, e2, rtol=1e-10)


def test_shifted_r_definition(rng):
    """shifted_r: (R^T R)[:p,:p] = A^T A + s I on the leading block with the
    stated shift; close to sketch_r by O(s / sigma_min^2); a rank-deficient
    sketch still has a finite factor (the shift keeps it positive definite)."""
    A = rng.standard_normal((50, 6))
    R = oracle.shifted_r(A, 5)
    G = A.T @ A
    s = 11.0 * (64 * 6 + 6 * 7) * 2.0 ** -53 * np.trace(G)   # 50 rows pad to 64
    np.testing.assert_allclose(R.T @ R, G[:5, :5] + s * np.eye(5), rtol=1e-13, atol=1e-12)
    Rq = oracle.sketch_r(A, 5)
    sig = np.linalg.svd(A[:, :5], compute_uv=False)
    assert np.abs(R - Rq).max() <= 10 * s / sig[-1] ** 2 * np.abs(Rq).max() + 1e-13 * np.abs(Rq).max()
    B = np.column_stack([A[:, 0], A[:, 0], A[:, 1]])   # exactly rank 2
    Rb = oracle.shifted_r(B, 3)
    assert np.all(np.isfinite(Rb)) and np.all(np.diag(Rb) > 0)
