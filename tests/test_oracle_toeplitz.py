"""Pins for oracle.toeplitz: the lag matrix of eq. (xphi) and the blocked
circulant-embedding layout, checked against a hand-written example and the
Toeplitz structure (Definition of a Toeplitz matrix), not against itself."""
import numpy as np
import pytest

import oracle
from tests.conftest import read_golden


def test_xphi_worked_example():
    y_s, p_s, X_s, b_s = read_golden("xphi_example.txt")
    y = np.array(y_s[0], dtype=float)
    p = int(p_s[0][0])
    X_expect = np.array(X_s, dtype=float)
    b_expect = np.array(b_s[0], dtype=float)
    X, b = oracle.lag_matrix(y, p)
    assert np.array_equal(X, X_expect)
    assert np.array_equal(b, b_expect)


@pytest.mark.parametrize("n,p", [(9, 1), (12, 4), (30, 7)])
def test_constant_descending_diagonals(n, p, rng):
    y = rng.standard_normal(n)
    X, b = oracle.lag_matrix(y, p)
    assert X.shape == (n - p, p)
    # constant along each descending diagonal
    for i in range(1, X.shape[0]):
        assert np.array_equal(X[i, 1:], X[i - 1, :-1])
    # the response is the next value after row i's first lag
    assert np.array_equal(b[:-1], X[1:, 0])
    # only n - 1 distinct numbers: y_0..y_{n-2} appear in X, y_n-1 only in b
    assert set(X.ravel()) == set(y[:-1])


@pytest.mark.parametrize("n,p,B", [(40, 3, 8), (64, 5, 16), (100, 17, 32), (33, 1, 4)])
def test_block_windows_reconstruct_rows(n, p, B, rng):
    """Every row of X sits inside its block's window at the stated offsets."""
    y = rng.standard_normal(n)
    X, _ = oracle.lag_matrix(y, p)
    W = oracle.block_windows(y, p, B)
    L = B - p + 1
    for i in range(n - p):
        k, r = divmod(i, L)
        row = W[k, r + p - 1 - np.arange(p)]
        assert np.array_equal(row, X[i])


def test_block_matvec_equals_dense(rng):
    """Overlap-save convolution with the block spectra reproduces X v and
    X^T u (exact identity; FP64 to 1e-13 relative on tiny sizes)."""
    for n in range(6, 65, 7):
        for p in range(1, n // 2 + 1):
            y = rng.standard_normal(n)
            v = rng.standard_normal(p)
            u = rng.standard_normal(n - p)
            X, _ = oracle.lag_matrix(y, p)
            B = 1
            while B < 2 * p:
                B *= 2
            Yb = oracle.block_spectra(y, p, B)
            L = B - p + 1
            vh = np.fft.rfft(np.concatenate([v, np.zeros(B - p)]))
            xv = np.concatenate([np.fft.irfft(Yb[k] * vh, B)[p - 1:] for k in range(Yb.shape[0])])[: n - p]
            assert np.allclose(xv, X @ v, rtol=0, atol=1e-13 * np.abs(y).max() * np.abs(v).sum())
            g = np.zeros(p)
            for k in range(Yb.shape[0]):
                z = np.zeros(B)
                seg = u[k * L: (k + 1) * L]
                z[p - 1: p - 1 + seg.size] = seg
                g += np.fft.irfft(np.conj(Yb[k]) * np.fft.rfft(z), B)[:p]
            assert np.allclose(g, X.T @ u, rtol=0, atol=1e-13 * np.abs(y).max() * np.abs(u).sum())
