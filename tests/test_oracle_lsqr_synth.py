"""Pins for oracle.lsqr (converged iterate vs the QR oracle; exact one-step
convergence with an exact preconditioner) and for the synthetic generator
(determinism, stationarity, recovery of the generating coefficients)."""
import numpy as np
import pytest

import oracle
import synth


def test_lsqr_converges_to_qr_solution(rng):
    for p in (1, 3, 10):
        y = synth.ar_series(4000, p, rng, 0.3, 0.9)
        X, _ = oracle.lag_matrix(y, p)
        idx, sc = oracle.uniform_rows(rng.random(20 * p), X.shape[0])
        S = oracle.sketch_rows(y, p, idx, sc)
        R = oracle.qr_r(S[:, :p])
        out = oracle.lsqr(y, p, oracle.tri_inverse(R), tol=1e-12)
        ref = oracle.fit_qr(y, p)
        assert out["istop"] in (1, 2)
        assert oracle.rel_error(out["phi"], ref["phi"]) < 1e-9 * max(1.0, ref["kappa"])


def test_lsqr_exact_preconditioner_one_step(rng):
    """With M = R^{-1} from the QR of X itself, A = X M has orthonormal
    columns, so the Krylov space is spanned after one step."""
    y = synth.ar_series(3000, 6, rng, 0.3, 0.9)
    X, _ = oracle.lag_matrix(y, 6)
    R = oracle.qr_r(X)
    out = oracle.lsqr(y, 6, oracle.tri_inverse(R), tol=1e-10)
    assert out["iters"] <= 2
    assert oracle.rel_error(out["phi"], oracle.fit_qr(y, 6)["phi"]) < 1e-12


def test_lsqr_warm_start_at_solution(rng):
    y = synth.ar_series(2000, 4, rng, 0.3, 0.9)
    ref = oracle.fit_qr(y, 4)
    out = oracle.lsqr(y, 4, oracle.tri_inverse(ref["R"]), phi0=ref["phi"], tol=1e-8)
    assert out["iters"] <= 1
    assert oracle.rel_error(out["phi"], ref["phi"]) < 1e-12


def test_generator_deterministic():
    a = synth.workload_ar100(seed=3, n=5000).y
    b = synth.workload_ar100(seed=3, n=5000).y
    c = synth.workload_ar100(seed=4, n=5000).y
    assert a.tobytes() == b.tobytes()
    assert a.tobytes() != c.tobytes()


def test_ar3_stationary_variance():
    """Sample variance of the AR(3) workload matches the process variance
    sum_k psi_k^2 (psi = MA(infinity) weights of the recursion) within 5%."""
    f = synth.workload_ar3(seed=0, n=200_000)
    phi = np.array(synth.workloads.AR3_PHI)
    psi = np.zeros(400)
    psi[0] = 1.0
    for k in range(1, 400):
        psi[k] = sum(phi[j] * psi[k - 1 - j] for j in range(3) if k - 1 - j >= 0)
    assert abs(f.y.var() / np.sum(psi ** 2) - 1) < 0.05


def test_cascade_matches_direct_recursion(rng):
    """The biquad cascade is the same filter as the direct AR recursion with
    coefficients from the poles (small p, where the direct form is stable)."""
    y, poles = synth.ar_series(3000, 5, np.random.default_rng(9), 0.3, 0.8, burn=0,
                               return_poles=True)
    phi = synth.poles_to_coefficients(*poles)
    rng2 = np.random.default_rng(9)
    synth.ar.draw_poles(rng2, 5, 0.3, 0.8)
    x = rng2.standard_normal(3000)
    yd = np.zeros(3000)
    for t in range(3000):
        acc = x[t]
        for j in range(5):
            if t - 1 - j >= 0:
                acc += phi[j] * yd[t - 1 - j]
        yd[t] = acc
    assert np.allclose(y, yd, atol=1e-10)


def test_fit_recovers_generating_coefficients():
    """OLS on a long AR(3) series lands within sampling error of the truth."""
    f = synth.workload_ar3(seed=0, n=200_000)
    phi = oracle.fit_qr(f.y, 3)["phi"]
    assert np.allclose(phi, synth.workloads.AR3_PHI, atol=0.01)


def test_outliers_recipe(rng):
    y = np.zeros(2000)
    z = synth.add_outliers(y, rng, 100)
    assert np.count_nonzero(z) == 100


def test_batch_and_serve_shapes():
    fits = synth.workload_batch(seed=0, count=16)
    for f in fits:
        assert 2 ** 12 - 1 <= f.y.size <= 2 ** 18 + 1
        assert 4 <= f.p <= 64
    t, which, pool = synth.workload_serve(seed=0, rate=100, duration=1.0, pool=4, hi_exp=12)
    assert np.all(np.diff(t) > 0) and t[-1] < 1.0
    assert which.max() < 4 and len(pool) == 4
