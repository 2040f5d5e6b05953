"""ctypes loader for liblrinv.so (the C ABI in include/lrinv.h).

Marshalling only: no arithmetic of the method happens in Python. Importing the
package without the built library raises immediately; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblrinv.so")

(LR_OK, LR_ERR_ARG, LR_ERR_SHAPE, LR_ERR_NOT_POW2, LR_ERR_WORKSPACE, LR_ERR_HIP, LR_ERR_UNSUPPORTED,
 LR_ERR_SCRATCH_LIMIT) = range(8)
NOALLOC_SCRATCH_BYTES = 32 << 20
LR_KERNEL_SE, LR_KERNEL_MATERN32 = 0, 1
LR_OMEGA_SRHT, LR_OMEGA_GAUSS = 0, 1
LR_PREC_F64, LR_PREC_F32, LR_PREC_BF16, LR_PREC_BF16X2 = 0, 1, 2, 3
LR_TRANSFORM_DCT, LR_TRANSFORM_DHT, LR_TRANSFORM_WHT = 0, 1, 2
TRANSFORMS = {"dct": LR_TRANSFORM_DCT, "dht": LR_TRANSFORM_DHT, "wht": LR_TRANSFORM_WHT}

PRECS = {"f64": LR_PREC_F64, "f32": LR_PREC_F32, "bf16": LR_PREC_BF16, "bf16x2": LR_PREC_BF16X2}
KERNELS = {"se": LR_KERNEL_SE, "matern32": LR_KERNEL_MATERN32}

c_i32, c_i64, c_dbl, c_vp, c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class LrHyper(ctypes.Structure):
    _fields_ = [("kernel", c_i32), ("reserved", c_i32), ("ell", c_dbl), ("s", c_dbl)]


class LrOmega(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("d", c_i32), ("n", c_i64), ("ld", c_i64),
                ("signs", c_vp), ("cols", c_vp), ("dense_t", c_vp)]


class LrError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}")


_SIGS = {
    "lr_version": (c_i32, []),
    "lr_status_string": (ctypes.c_char_p, [c_i32]),
    "lr_check_srht_cols": (c_i32, [c_vp, c_i32, c_i64]),
    "lr_structured_omega": (c_i32, [c_vp, c_i32, c_i64, c_i32, c_vp, c_vp, c_i32, c_vp, c_i64]),
    "lr_sketch_workspace_bytes": (c_sz, [c_i64, c_i32, c_i32, c_i32]),
    "lr_sketch": (c_i32, [c_vp, c_i64, c_i32, c_vp, ctypes.POINTER(LrHyper), ctypes.POINTER(LrOmega), c_dbl, c_i32,
                          c_vp, c_vp, c_vp, c_sz]),
    "lr_sketch_noalloc": (c_i32, [c_vp, c_i64, c_i32, c_vp, ctypes.POINTER(LrHyper), ctypes.POINTER(LrOmega), c_dbl,
                                  c_i32, c_vp, c_vp]),
    "lr_sketch_grid_workspace_bytes": (c_sz, [c_i64, c_i32, c_i32, c_i32]),
    "lr_sketch_grid": (c_i32, [c_vp, c_i64, c_i32, c_vp, c_i32, c_vp, ctypes.POINTER(LrOmega), c_dbl, c_i32, c_vp,
                               c_vp, c_sz]),
    "lr_tsqr_workspace_bytes": (c_sz, [c_i64, c_i32, c_i32, c_i32]),
    "lr_tsqr": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_sz]),
    "lr_tsqr_tree_workspace_bytes": (c_sz, [c_i64, c_i32, c_i32, c_i32, c_i32]),
    "lr_tsqr_tree": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_sz]),
    "lr_lowrank_solve_workspace_bytes": (c_sz, [c_i64, c_i32, c_i32, c_i32]),
    "lr_lowrank_solve": (c_i32, [c_vp, c_i64, c_i32, c_i32, ctypes.POINTER(LrOmega), c_i32, c_vp, c_vp, c_dbl, c_dbl,
                                 c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz]),
    "lr_loglik": (c_i32, [c_vp, c_i64, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lr_projection_solve_workspace_bytes": (c_sz, [c_i64, c_i32, c_i32, c_i32, c_i32]),
    "lr_projection_solve": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_vp, ctypes.POINTER(LrHyper), c_i32, c_vp, c_dbl,
                                    c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz]),
    "lr_psd_part_workspace_bytes": (c_sz, [c_i32]),
    "lr_psd_part": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_sz]),
    "lr_backward_workspace_bytes": (c_sz, [c_i64, c_i32, c_i32, c_i32, c_i32]),
    "lr_backward": (c_i32, [c_vp, c_i64, c_i32, c_vp, ctypes.POINTER(LrHyper), ctypes.POINTER(LrOmega), c_i32, c_vp,
                            c_vp, c_vp, c_vp, c_vp, c_vp, c_dbl, c_dbl, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp,
                            c_vp, c_sz]),
}

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1312_1869_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def status_string(status: int) -> str:
    try:
        return lib().lr_status_string(int(status)).decode()
    except ImportError:
        return f"status {status}"


def check(status: int, where: str) -> None:
    if status != LR_OK:
        raise LrError(int(status), where)
