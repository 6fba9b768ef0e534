"""OLS solution of the Toeplitz AR(p) problem by dense QR (oracle; test
infrastructure only).

Definition 2.1 (OLS problem) and Theorem 2.2 (its solution): the minimiser of
||A x - b||^2 satisfies the normal equations A^T A x = A^T b; it is unique
when A^T A is nonsingular, otherwise the minimum-norm solution comes from the
SVD of A.  Section 2.1 names QR factorisation as the conventional direct
method for a least-squares problem.

fit_qr forms [X | b] of eq. (xphi) densely and calls LAPACK's Householder QR
(dgeqrf through scipy.linalg.qr): with [X | b] = Q R_A,

    phi* = R_A[:p,:p]^{-1} R_A[:p, p],   ||b - X phi*|| = |R_A[p, p]|.

fit_svd is the minimum-norm solution (LAPACK gelsd) of Theorem 2.2's
singular case; householder_qr is a hand-written Householder QR used only to
cross-check LAPACK on small inputs.

Parity pins (tests/test_oracle_ols.py): exact rational solutions of the normal
equations by brute-force enumeration of every series in {-1,0,1}^n, n <= 7,
p <= 3; the p = 1 closed form; exact recovery on noise-free AR recursions;
normal-equation orthogonality; LAPACK vs hand-written Householder vs SVD.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .toeplitz import lag_matrix


def qr_r(A) -> np.ndarray:
    """Upper-triangular R of A = QR by LAPACK dgeqrf (economic, n_cols x n_cols)."""
    A = np.asarray(A, dtype=np.float64)
    R = sla.qr(A, mode="r", check_finite=True)[0]
    k = min(A.shape)
    return np.triu(R[:k, :])


def fit_qr(y, p: int) -> dict:
    """phi*, ||r*||, R and kappa(X) by Householder QR of [X | b] (module doc)."""
    X, b = lag_matrix(y, p)
    RA = qr_r(np.column_stack([X, b]))
    R = RA[:p, :p]
    q = RA[:p, p]
    phi = sla.solve_triangular(R, q, lower=False)
    rnorm = abs(RA[p, p]) if RA.shape[0] > p else 0.0
    return {"phi": phi, "rnorm": float(rnorm), "R": R, "kappa": kappa(R)}


def fit_svd(X, b) -> np.ndarray:
    """Minimum-norm least-squares solution (Theorem 2.2, singular case)."""
    x, *_ = np.linalg.lstsq(np.asarray(X, np.float64), np.asarray(b, np.float64), rcond=None)
    return x


def householder_qr(A):
    """Plain Householder QR, one column at a time: returns (Q, R) with A = Q R,
    Q with orthonormal columns (n x k), R upper triangular (k x k)."""
    A = np.array(A, dtype=np.float64, copy=True)
    n, k = A.shape
    Q = np.eye(n)
    for j in range(min(k, n)):
        x = A[j:, j]
        normx = np.sqrt(np.sum(x * x))
        if normx == 0.0:
            continue
        alpha = -normx if x[0] >= 0 else normx
        v = x.copy()
        v[0] -= alpha
        vnorm2 = np.sum(v * v)
        if vnorm2 == 0.0:
            continue
        # A <- (I - 2 v v^T / v^T v) A on rows j..n-1
        for c in range(j, k):
            A[j:, c] -= (2.0 * np.dot(v, A[j:, c]) / vnorm2) * v
        for r in range(n):
            Q[r, j:] -= (2.0 * np.dot(Q[r, j:], v) / vnorm2) * v
    R = np.triu(A[:k, :])
    return Q[:, :k], R


def kappa(R) -> float:
    """2-norm condition number sigma_max / sigma_min from the singular values
    of the triangular factor (equal to those of X)."""
    s = np.linalg.svd(np.asarray(R, np.float64), compute_uv=False)
    if s[-1] == 0.0:
        return float("inf")
    return float(s[0] / s[-1])


def rel_error(phi_hat, phi) -> float:
    """||phi_hat - phi|| / ||phi||: eq. (phierr) without the factor 100."""
    phi_hat = np.asarray(phi_hat, np.float64)
    phi = np.asarray(phi, np.float64)
    return float(np.linalg.norm(phi_hat - phi) / np.linalg.norm(phi))


def residual_norm(y, p: int, phi) -> float:
    """||b - X phi|| with X, b formed densely."""
    X, b = lag_matrix(y, p)
    return float(np.linalg.norm(b - X @ np.asarray(phi, np.float64)))


def normal_residual(y, p: int, phi) -> float:
    """||X^T r|| / (||X||_2 ||r||) for r = b - X phi: zero at the OLS solution
    by Theorem 2.2's normal equations."""
    X, b = lag_matrix(y, p)
    r = b - X @ np.asarray(phi, np.float64)
    return float(np.linalg.norm(X.T @ r) / (np.linalg.norm(X, 2) * np.linalg.norm(r)))


def tri_inverse(R) -> np.ndarray:
    """R^{-1} for upper-triangular R by back-substitution on the identity."""
    R = np.asarray(R, np.float64)
    return sla.solve_triangular(R, np.eye(R.shape[0]), lower=False)
