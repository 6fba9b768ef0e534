"""Shared helpers of the GPU parity tests (device tensors through torch, calls
through the C-ABI binding).  Imported only by tests marked `gpu`."""
import math
import sys

import numpy as np

EPS64 = 2.0 ** -53
EPS32 = 2.0 ** -24


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def capi():
    from paper_2112_12994_amd import capi as c
    return c


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm device")
    return torch, torch.device("cuda", 0)


def to_dev(a, dtype=None):
    torch, dev = torch_dev()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def unpack_spectra(packed: np.ndarray, B: int) -> np.ndarray:
    """Packed block spectra (nblocks x B/2 complex words) -> (nblocks, B/2+1) bins."""
    N = B // 2
    out = np.zeros((packed.shape[0], N + 1), dtype=np.complex128)
    out[:, 1:N] = packed[:, 1:N]
    out[:, 0] = packed[:, 0].real
    out[:, N] = packed[:, 0].imag
    return out


def fft_tol(eps, B, scale):
    """Error bound used for one blocked FFT product: C eps log2(B) * scale."""
    return 16.0 * eps * math.log2(B) * scale


def chunked_matvec_norms(y, p, d, phi, step=1 << 18):
    """(||X d||, ||X phi||) with the oracle's dense products on row chunks."""
    import oracle
    m = y.size - p
    a2 = b2 = 0.0
    for a in range(0, m, step):
        rows = min(step, m - a)
        seg = y[a: a + rows + p]
        a2 += float(np.sum(oracle.matvec(seg, p, d) ** 2))
        b2 += float(np.sum(oracle.matvec(seg, p, phi) ** 2))
    return math.sqrt(a2), math.sqrt(b2)


def attainable(phi, rnorm, kappa, smax, xphi_norm, b_norm, p, B, tol):
    """Accuracy an FP64 solve can reach (least-squares perturbation theory to
    first order, e.g. Higham, Accuracy and Stability of Numerical Algorithms,
    ch. 20).  The solve is backward stable with normwise backward error
    eta = 16 eps log2(B) (one blocked FFT product) + tol (LSQR's stopping
    test bounds the normal-equation residual relative to ||A|| ||r||):
      coefficients   eta kappa + eta kappa^2 ||r|| / (||X|| ||phi||)
      fitted values  eta (kappa ||r|| + ||X|| ||phi|| + ||b||) / ||X phi||
    """
    eta = 16 * EPS64 * math.log2(B) + tol
    phin = float(np.linalg.norm(phi))
    coef = eta * kappa + eta * kappa ** 2 * rnorm / (smax * phin)
    fit = eta * (kappa * rnorm + smax * phin + b_norm) / xphi_norm
    return coef, fit


def resid_tol(phi, rnorm, smax, y_max, p, xdphi_norm):
    """Bound on | ||r(phi_hat)|| - ||r*|| |: the second-order change at the
    minimiser, ||X dphi||^2 / (2 ||r*||) (dphi measured), plus the rounding of
    the residual rows themselves (each a p-term dot product: 4 sqrt(p) eps
    max|y| (1 + ||phi||_1), errors uncorrelated with r) and of the oracle's
    own |R[p,p]| (16 eps ||X||)."""
    second = xdphi_norm ** 2 / (2 * rnorm) if rnorm > 0 else xdphi_norm
    return 1.01 * second + 4 * math.sqrt(p) * EPS64 * y_max * (1 + float(np.abs(phi).sum())) \
        + 16 * EPS64 * smax
