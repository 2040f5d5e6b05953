"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/lrinv.h, and rejects bad arguments on the host before any
launch (every call below fails validation, so no device is touched)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1312_1869_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: validation fails first


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lrinv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lr_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) >= set(L._SIGS)


def test_version_and_status_strings():
    lib = L.lib()
    assert lib.lr_version() >> 16 == 2 and lib.lr_version() & 0xFFFF >= 1
    assert lib.lr_status_string(L.LR_ERR_NOT_POW2) == b"LR_ERR_NOT_POW2"
    assert lib.lr_status_string(99) == b"LR_UNKNOWN_STATUS"


def test_check_srht_cols():
    lib = L.lib()
    ok = np.array([0, 3, 9, 1023], dtype=np.int32)
    dup = np.array([0, 3, 3], dtype=np.int32)
    out = np.array([0, 1024], dtype=np.int32)
    neg = np.array([-1, 2], dtype=np.int32)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert lib.lr_check_srht_cols(p(ok), 4, 1024) == L.LR_OK
    assert lib.lr_check_srht_cols(p(dup), 3, 1024) == L.LR_ERR_ARG
    assert lib.lr_check_srht_cols(p(out), 2, 1024) == L.LR_ERR_ARG
    assert lib.lr_check_srht_cols(p(neg), 2, 1024) == L.LR_ERR_ARG


def _hyper(kernel=L.LR_KERNEL_SE, ell=0.2, s=1.0, reserved=0):
    return L.LrHyper(kernel, reserved, ell, s)


def _srht(n, d):
    return L.LrOmega(L.LR_OMEGA_SRHT, d, n, 0, FAKE, FAKE, None)


def _gauss(n, d, ld):
    return L.LrOmega(L.LR_OMEGA_GAUSS, d, n, ld, None, None, FAKE)


def _sketch(n=1024, D=2, hyp=None, om=None, nu=0.0, prec=L.LR_PREC_F32, ws_bytes=1 << 30, y=FAKE, yp=None):
    lib = L.lib()
    hyp = hyp if hyp is not None else _hyper()
    om = om if om is not None else _srht(n, 64)
    return lib.lr_sketch(None, n, D, FAKE, ctypes.byref(hyp), ctypes.byref(om), nu, prec, y, yp,
                         ctypes.c_void_p(0x100000), ws_bytes)


def test_sketch_validation():
    assert _sketch(n=1000, om=_srht(1000, 64)) == L.LR_ERR_NOT_POW2
    assert _sketch(prec=L.LR_PREC_BF16) == L.LR_ERR_UNSUPPORTED
    assert _sketch(prec=7) == L.LR_ERR_ARG
    assert _sketch(hyp=_hyper(ell=float("nan"))) == L.LR_ERR_ARG
    assert _sketch(hyp=_hyper(ell=0.0)) == L.LR_ERR_ARG
    assert _sketch(hyp=_hyper(s=-1.0)) == L.LR_ERR_ARG
    assert _sketch(hyp=_hyper(kernel=5)) == L.LR_ERR_ARG
    assert _sketch(hyp=_hyper(reserved=1)) == L.LR_ERR_ARG
    assert _sketch(nu=float("inf")) == L.LR_ERR_ARG
    assert _sketch(D=0) == L.LR_ERR_SHAPE
    assert _sketch(D=16) == L.LR_ERR_SHAPE
    assert _sketch(om=_srht(1024, 2048)) == L.LR_ERR_SHAPE
    assert _sketch(om=_srht(512, 64)) == L.LR_ERR_SHAPE  # omega->n != n
    assert _sketch(om=_gauss(1000, 64, 1001), n=1000) == L.LR_ERR_SHAPE  # ld % 8
    assert _sketch(om=_gauss(1000, 64, 992), n=1000) == L.LR_ERR_SHAPE  # ld < n
    big = (1 << 25) + 8
    assert _sketch(om=_gauss(big, 64, big), n=big, prec=L.LR_PREC_BF16) == L.LR_ERR_UNSUPPORTED  # bf16 n > 2^25
    assert _sketch(y=None, yp=None) == L.LR_ERR_ARG
    assert _sketch(ws_bytes=16) == L.LR_ERR_WORKSPACE


def test_tsqr_validation():
    lib = L.lib()
    ws = ctypes.c_void_p(0x100000)
    t = lambda n, d, leaf, prec=L.LR_PREC_F32, wsb=1 << 40: lib.lr_tsqr(None, n, d, leaf, prec, FAKE, FAKE, FAKE, ws, wsb)
    assert t(4096, 64, 32) == L.LR_ERR_SHAPE       # leaf_rows < d
    assert t(4096, 64, 16384) == L.LR_ERR_SHAPE    # leaf_rows > 8192
    assert t(4100, 64, 1024) == L.LR_ERR_SHAPE     # last leaf 4 < d
    assert t(60, 64, 64) == L.LR_ERR_SHAPE         # d > n
    assert t(4096, 2000, 4096) == L.LR_ERR_SHAPE   # d > 1024
    assert t(4096, 64, 1024, wsb=100) == L.LR_ERR_WORKSPACE
    assert lib.lr_tsqr(None, 4096, 64, 1024, L.LR_PREC_F32, FAKE, FAKE, FAKE, ctypes.c_void_p(0x100010),
                       1 << 40) == L.LR_ERR_WORKSPACE  # misaligned workspace
    assert lib.lr_tsqr_workspace_bytes(4096, 64, 1024, L.LR_PREC_F32) > 4096 * 64 * 4
    assert lib.lr_tsqr_workspace_bytes(4096, 64, 32, L.LR_PREC_F32) == 0


def test_solve_and_backward_validation():
    lib = L.lib()
    om = _srht(1024, 64)
    ws = ctypes.c_void_p(0x100000)
    s = lambda sigma2=1e-3, nu=0.0, m=4, A=FAKE, X=ctypes.c_void_p(0x20000), wsb=1 << 40, prec=L.LR_PREC_F32: \
        lib.lr_lowrank_solve(None, 1024, 64, m, ctypes.byref(om), prec, FAKE, FAKE, sigma2, nu, A, X, FAKE, FAKE, FAKE,
                             FAKE, FAKE, FAKE, ws, wsb)
    assert s(sigma2=0.0) == L.LR_ERR_ARG
    assert s(sigma2=-1.0) == L.LR_ERR_ARG
    assert s(nu=-0.1) == L.LR_ERR_ARG
    assert s(m=65) == L.LR_ERR_SHAPE
    assert s(A=FAKE, X=FAKE) == L.LR_ERR_ARG      # X aliases A
    assert s(wsb=8) == L.LR_ERR_WORKSPACE
    assert s(prec=L.LR_PREC_BF16) == L.LR_ERR_UNSUPPORTED
    hyp = _hyper()
    b = lambda mode=0, m=1, sigma2=1e-3, nu=0.0, R=FAKE: lib.lr_backward(
        None, 1024, 2, FAKE, ctypes.byref(hyp), ctypes.byref(om), L.LR_PREC_F32, FAKE, R, FAKE, FAKE, FAKE, FAKE,
        sigma2, nu, mode, m, FAKE, FAKE, None, FAKE, None, ws, 1 << 40)
    assert b(mode=2) == L.LR_ERR_ARG
    assert b(mode=0, m=2) == L.LR_ERR_SHAPE
    assert b(sigma2=float("nan")) == L.LR_ERR_ARG
    assert b(nu=-1e-3) == L.LR_ERR_ARG
    assert b(nu=1e-4, R=None) == L.LR_ERR_ARG     # a shift needs R
    assert lib.lr_loglik(None, 0, L.LR_PREC_F32, FAKE, FAKE, FAKE, None, FAKE) == L.LR_ERR_SHAPE


def test_structured_omega_validation():
    lib = L.lib()
    so = lambda t=L.LR_TRANSFORM_DCT, n=1000, d=64, prec=L.LR_PREC_F32, ld=1008, out=FAKE, signs=FAKE: \
        lib.lr_structured_omega(None, t, n, d, signs, FAKE, prec, out, ld)
    assert so(t=3) == L.LR_ERR_ARG
    assert so(prec=9) == L.LR_ERR_ARG
    assert so(ld=1001) == L.LR_ERR_SHAPE          # ld % 8
    assert so(ld=992) == L.LR_ERR_SHAPE           # ld < n
    assert so(d=2000, n=4096, ld=4096) == L.LR_ERR_SHAPE  # d > 1024
    assert so(d=0) == L.LR_ERR_SHAPE
    assert so(t=L.LR_TRANSFORM_WHT) == L.LR_ERR_NOT_POW2  # n = 1000
    assert so(out=None) == L.LR_ERR_ARG
    assert so(out=ctypes.c_void_p(0x10008)) == L.LR_ERR_ARG  # not 16-byte aligned
    assert so(signs=None) == L.LR_ERR_ARG


def test_sketch_grid_validation():
    lib = L.lib()
    hs = (L.LrHyper * 3)(_hyper(ell=0.2), _hyper(ell=0.3), _hyper(ell=0.4))
    mixed = (L.LrHyper * 2)(_hyper(), _hyper(kernel=L.LR_KERNEL_MATERN32))
    bad = (L.LrHyper * 2)(_hyper(), _hyper(ell=-1.0))
    om = _srht(1024, 64)
    ws = ctypes.c_void_p(0x100000)
    g = lambda hyps=hs, nt=3, n=1024, o=om, prec=L.LR_PREC_F32, nu=0.0, y=FAKE, wsb=1 << 30: lib.lr_sketch_grid(
        None, n, 2, FAKE, nt, ctypes.cast(hyps, ctypes.c_void_p), ctypes.byref(o), nu, prec, y, ws, wsb)
    assert g(nt=0) == L.LR_ERR_SHAPE
    assert g(nt=5000) == L.LR_ERR_SHAPE
    assert g(hyps=mixed, nt=2) == L.LR_ERR_ARG     # one kernel kind per grid
    assert g(hyps=bad, nt=2) == L.LR_ERR_ARG
    assert g(nu=-1.0) == L.LR_ERR_ARG
    assert g(y=None) == L.LR_ERR_ARG
    assert g(prec=L.LR_PREC_BF16) == L.LR_ERR_UNSUPPORTED  # bf16 with SRHT
    assert g(n=1000, o=_srht(1000, 64)) == L.LR_ERR_NOT_POW2
    assert g(wsb=16) == L.LR_ERR_WORKSPACE
    assert lib.lr_sketch_grid_workspace_bytes(1024, 2, 64, L.LR_PREC_F32) == \
        lib.lr_sketch_workspace_bytes(1024, 2, 64, L.LR_PREC_F32)


def test_projection_and_psd_validation():
    lib = L.lib()
    hyp = _hyper()
    ws = ctypes.c_void_p(0x100000)
    pj = lambda n=4096, d=64, m=2, prec=L.LR_PREC_F32, sigma2=1e-3, clip=1, A=FAKE, X=ctypes.c_void_p(0x20000), \
        wsb=1 << 40, D=2: lib.lr_projection_solve(None, n, D, d, FAKE, ctypes.byref(hyp), prec, FAKE, sigma2, clip, m,
                                                  A, X, FAKE, FAKE, FAKE, FAKE, ws, wsb)
    assert pj(clip=2) == L.LR_ERR_ARG
    assert pj(sigma2=0.0) == L.LR_ERR_ARG
    assert pj(prec=5) == L.LR_ERR_ARG
    assert pj(d=2048) == L.LR_ERR_SHAPE
    assert pj(d=5000, n=4096) == L.LR_ERR_SHAPE
    assert pj(m=65) == L.LR_ERR_SHAPE
    assert pj(D=16) == L.LR_ERR_SHAPE
    assert pj(A=FAKE, X=FAKE) == L.LR_ERR_ARG
    assert pj(wsb=64) == L.LR_ERR_WORKSPACE
    assert lib.lr_projection_solve_workspace_bytes(4096, 2, 64, 2, L.LR_PREC_F32) > 4096 * 64 * 8
    assert lib.lr_psd_part(None, 0, FAKE, FAKE, ws, 1 << 30) == L.LR_ERR_SHAPE
    assert lib.lr_psd_part(None, 2000, FAKE, FAKE, ws, 1 << 30) == L.LR_ERR_SHAPE
    assert lib.lr_psd_part(None, 64, FAKE, FAKE, ws, 1 << 30) == L.LR_ERR_ARG  # Bplus aliases B
    assert lib.lr_psd_part(None, 64, FAKE, ctypes.c_void_p(0x30000), ws, 8) == L.LR_ERR_WORKSPACE
    assert lib.lr_psd_part_workspace_bytes(64) >= 3 * 64 * 64 * 8


def test_tsqr_tree_validation():
    lib = L.lib()
    ws = ctypes.c_void_p(0x100000)
    t = lambda n=4096, d=64, leaf=512, group=2, prec=L.LR_PREC_F32, q=FAKE, wsb=1 << 40: lib.lr_tsqr_tree(
        None, n, d, leaf, group, prec, FAKE, q, FAKE, ws, wsb)
    assert t(group=0) == L.LR_ERR_SHAPE
    assert t(group=3) == L.LR_ERR_SHAPE           # 8 blocks are not a multiple of 3
    assert t(n=4100) == L.LR_ERR_SHAPE            # groups need whole blocks
    assert t(leaf=8192, n=16384, d=64) == L.LR_ERR_SHAPE  # d + leaf_rows > 8192 in a sequential step
    assert t(wsb=64) == L.LR_ERR_WORKSPACE
    assert t(group=1, n=4160, wsb=64) == L.LR_ERR_WORKSPACE  # the binary tree takes a short last block
    assert lib.lr_tsqr_tree_workspace_bytes(4096, 64, 512, 1, L.LR_PREC_F32) == \
        lib.lr_tsqr_workspace_bytes(4096, 64, 512, L.LR_PREC_F32)
    assert lib.lr_tsqr_tree_workspace_bytes(4096, 64, 512, 3, L.LR_PREC_F32) == 0
