"""Dense Toeplitz lag matrix and its products (oracle; test infrastructure only).

Section 3, eq. (xphi): regressing y_t on its p lags gives the (n-p) x p data
matrix whose row t holds (y_{t-1}, ..., y_{t-p}) and the response y_t, for
t = p+1..n (1-based).  With 0-based indices, m = n - p rows:

    X[i, j] = y[p - 1 + i - j],   b[i] = y[p + i],   i in [0, m), j in [0, p).

X is Toeplitz (Definition of a Toeplitz matrix: constant descending
diagonals), so it holds only n - 1 distinct values (Section 3, the remark
after eq. (TOLS)).

The products here form X densely and multiply: the plain definitions that the
FFT matvecs must reproduce.  Parity pins: the worked example fixture and the
structure checks in tests/test_oracle_toeplitz.py.

block_windows / block_spectra state the blocked circulant-embedding layout the
GPU path uses to apply X (not a construct of the paper, which only notes the
n + p - 1 distinct values): block k covers rows [k*L, k*L + L) with L = B - p + 1
and holds the window y[k*L : k*L + B] (zero past the end of y); its spectrum is
the length-B real DFT of that window.
"""
from __future__ import annotations

import numpy as np


def lag_matrix(y, p: int):
    """(X, b) of eq. (xphi), 0-based as in the module docstring."""
    y = np.asarray(y, dtype=np.float64)
    n = y.size
    if p < 1 or n < p + 1:
        raise ValueError("need p >= 1 and n >= p + 1")
    m = n - p
    X = np.empty((m, p), dtype=np.float64)
    for j in range(p):
        X[:, j] = y[p - 1 - j: p - 1 - j + m]
    b = y[p:].copy()
    return X, b


def matvec(y, p: int, v) -> np.ndarray:
    """X v with X formed densely."""
    X, _ = lag_matrix(y, p)
    return X @ np.asarray(v, dtype=np.float64)


def rmatvec(y, p: int, u) -> np.ndarray:
    """X^T u with X formed densely."""
    X, _ = lag_matrix(y, p)
    return X.T @ np.asarray(u, dtype=np.float64)


def block_windows(y, p: int, B: int) -> np.ndarray:
    """Windows of the blocked layout (module docstring): shape (nblocks, B)."""
    y = np.asarray(y, dtype=np.float64)
    n = y.size
    m = n - p
    L = B - p + 1
    if L < 1:
        raise ValueError("block length must exceed p - 1")
    nb = -(-m // L)
    W = np.zeros((nb, B), dtype=np.float64)
    for k in range(nb):
        seg = y[k * L: min(k * L + B, n)]
        W[k, :seg.size] = seg
    return W


def block_spectra(y, p: int, B: int) -> np.ndarray:
    """Length-B real DFT (B/2 + 1 bins) of every window: shape (nblocks, B/2+1)."""
    return np.fft.rfft(block_windows(y, p, B), axis=1)
