"""R-preconditioned LSQR in plain FP64 NumPy (oracle; test infrastructure only).

The paper solves the compressed problem of eq. (OLSc) directly; the solver
here instead uses the sketch's triangular factor R as a right preconditioner
and iterates on the full problem, so that it converges to the exact OLS
solution of Theorem 2.2.  The iteration is LSQR as published by Paige and
Saunders (ACM TOMS 8(1), 1982): Golub-Kahan bidiagonalisation of A = X M
(M = R^{-1}) started from the residual of a warm start phi0, with the QR
update of the bidiagonal by plane rotations.

Stopping (atol = btol = tol, no condition limit): stop when
||A^T r|| <= tol ||A|| ||r||  or  ||r|| <= tol ||r0|| + tol ||A|| ||z||,
with ||A|| the Frobenius estimate accumulated from the alphas and betas.

Parity status: the converged iterate is pinned by the QR oracle (the tests
check agreement on well-conditioned problems); the iteration count is
parity unpinned (it depends on rounding; only bounds are checked).
"""
from __future__ import annotations

import numpy as np

from .toeplitz import lag_matrix


def lsqr(y, p: int, M, phi0=None, tol: float = 1e-10, max_iter: int = 1000):
    """Solve min ||X phi - b|| with A = X M; returns dict(phi, iters, istop, rnorm_est)."""
    X, b = lag_matrix(y, p)
    M = np.asarray(M, np.float64)
    phi0 = np.zeros(p) if phi0 is None else np.asarray(phi0, np.float64)
    r0 = b - X @ phi0

    def A(v):
        return X @ (M @ v)

    def AT(u):
        return M.T @ (X.T @ u)

    z = np.zeros(p)
    u = r0.copy()
    beta = np.linalg.norm(u)
    bnorm = beta
    if beta == 0.0:
        return {"phi": phi0, "iters": 0, "istop": 0, "rnorm_est": 0.0}
    u /= beta
    v = AT(u)
    alpha = np.linalg.norm(v)
    if alpha == 0.0:
        return {"phi": phi0, "iters": 0, "istop": 0, "rnorm_est": beta}
    v /= alpha
    w = v.copy()
    phibar, rhobar = beta, alpha
    anorm2 = 0.0
    istop, itn = 0, 0
    rnorm = beta
    while itn < max_iter:
        itn += 1
        u = A(v) - alpha * u
        beta = np.linalg.norm(u)
        anorm2 += alpha * alpha + beta * beta
        if beta > 0.0:
            u /= beta
        v = AT(u) - beta * v
        alpha = np.linalg.norm(v)
        if alpha > 0.0:
            v /= alpha
        rho = np.hypot(rhobar, beta)
        c, s = rhobar / rho, beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi_k = c * phibar
        phibar = s * phibar
        z = z + (phi_k / rho) * w
        w = v - (theta / rho) * w
        rnorm = phibar
        arnorm = phibar * alpha * abs(c)
        anorm = np.sqrt(anorm2)
        znorm = np.linalg.norm(z)
        if arnorm <= tol * anorm * rnorm:
            istop = 2
            break
        if rnorm <= tol * bnorm + tol * anorm * znorm:
            istop = 1
            break
        if alpha == 0.0 or beta == 0.0:
            istop = 3
            break
    return {"phi": phi0 + M @ z, "iters": itn, "istop": istop, "rnorm_est": float(rnorm)}
