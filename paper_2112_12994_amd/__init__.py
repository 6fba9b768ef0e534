"""Toeplitz least squares for AR(p) fitting on AMD MI355X (gfx950).

The compute path lives in libtls.so (HIP kernels + C-ABI, include/tls.h);
`capi` is its ctypes binding.  Build with `python -m paper_2112_12994_amd.build`.
"""
import os

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libtls.so")


def load():
    """Import and return the binding module (raises if libtls.so is missing)."""
    from . import capi
    return capi
