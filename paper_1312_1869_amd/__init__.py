"""MI355X-native randomized low-rank inverse of huge covariance matrices.

Sketch Y = K Omega with K evaluated on the fly (Sec. 3.1-3.2), binary-tree
blocked QR of Y (Sec. 3.3), Woodbury-form application of the approximate
inverse and the Gaussian log-likelihood, plus a hand-written adjoint for the
kernel hyperparameters. All compute runs in liblrinv.so (HIP, gfx950); see
include/lrinv.h for the C ABI.
"""
from . import _lib  # noqa: F401

__all__ = ["api", "autograd", "build"]


def __getattr__(name):
    if name in ("api", "autograd"):
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
