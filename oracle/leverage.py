"""Leverage scores and generalised leverage scores (oracle; test
infrastructure only).

Definition 2.6 (leverage score): for A (n x d, rank d) the i-th score is the
i-th diagonal entry of the hat matrix A (A^T A)^{-1} A^T; the scores are
non-negative and sum to d (eq. (ldist) turns them into a distribution).

Section 3.1 gives the exact p = 1 scores of the AR lag matrix in closed form:
y_i^2 / sum_{t=1}^{n-1} y_t^2 for i = 1..n-1.

Definition 3.6 (generalised leverage score of row i of C with respect to B)
is C(i,:)^T (B^T B)^{-1} C(i,:) = ||B (B^T B)^{-1} C(i,:)||^2, and eq. (glev)
approximates it by ||G B (B^T B)^{-1} C(i,:)||^2 with a random Gaussian G of
O(log n) rows.  With B = Q_B R_B, B (B^T B)^{-1} C(i,:) = Q_B R_B^{-T} C(i,:),
so the same estimate is ||C(i,:)^T R_B^{-1} (G Q_B)^T||^2: a k-column product
of the data rows with Omega = R_B^{-1} Pi^T for a k x d random map Pi.
scores_from_omega states that product form directly: it is what the GPU's
score pass computes once Omega is given.

Parity pins (tests/test_oracle_leverage.py): scores sum to d; the p = 1
closed form; hat matrix vs QR route; Theorem 3.7 (generalised scores w.r.t.
a uniform row subsample bound the true scores from above); the eq. (glev)
identity between the G-form and the Omega-form.
"""
from __future__ import annotations

import numpy as np

from .toeplitz import lag_matrix


def leverage_scores_hat(A) -> np.ndarray:
    """diag(A (A^T A)^{-1} A^T) straight from Definition 2.6 (small n only)."""
    A = np.asarray(A, np.float64)
    H = A @ np.linalg.solve(A.T @ A, A.T)
    return np.diag(H).copy()


def leverage_scores(A) -> np.ndarray:
    """Definition 2.6 via a thin QR: the hat matrix is Q Q^T, so the i-th
    score is the squared norm of row i of Q."""
    A = np.asarray(A, np.float64)
    Q, _ = np.linalg.qr(A, mode="reduced")
    return np.sum(Q * Q, axis=1)


def ar1_leverage(y) -> np.ndarray:
    """Closed-form exact p = 1 scores of Section 3.1 (0-based: row i uses
    y[i], the denominator sums y[0..n-2]^2)."""
    y = np.asarray(y, np.float64)
    den = np.sum(y[:-1] ** 2)
    return y[:-1] ** 2 / den


def generalized_scores(C, B) -> np.ndarray:
    """Definition 3.6: C(i,:)^T (B^T B)^{-1} C(i,:) for every row i of C."""
    C = np.asarray(C, np.float64)
    B = np.asarray(B, np.float64)
    Ginv = np.linalg.inv(B.T @ B)
    return np.einsum("ij,jk,ik->i", C, Ginv, C)


def approx_generalized_scores(C, B, G) -> np.ndarray:
    """eq. (glev): ||G B (B^T B)^{-1} C(i,:)||^2 with G of shape (k, rows(B))."""
    C = np.asarray(C, np.float64)
    B = np.asarray(B, np.float64)
    G = np.asarray(G, np.float64)
    K = G @ B @ np.linalg.inv(B.T @ B)          # k x d
    Z = C @ K.T                                  # rows x k
    return np.sum(Z * Z, axis=1)


def scores_from_omega(y, p: int, Omega) -> np.ndarray:
    """sum_q (X Omega)[i, q]^2 for every row i of the lag matrix X."""
    X, _ = lag_matrix(y, p)
    Z = X @ np.asarray(Omega, np.float64)
    return np.sum(Z * Z, axis=1)
