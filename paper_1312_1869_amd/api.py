"""Torch-facing wrappers of the lrinv C ABI.

Tensors supply device memory and the current stream; every step of the method
runs in liblrinv.so. Functions mirror the C entry points:

* ``sketch``        Y = (K_f + nu I) Omega           (lr_sketch)
* ``tsqr``          Y = Q R, binary-tree blocked QR  (lr_tsqr)
* ``lowrank_solve`` K~^{-1} A, log|K~|, factors      (lr_lowrank_solve)
* ``loglik``        -1/2 y^T alpha - 1/2 log|K~|      (lr_loglik)
* ``backward``      d/d(log ell, log s, log sigma2)  (lr_backward)
"""
from __future__ import annotations

import ctypes
import dataclasses
import math

import numpy as np
import torch

from . import _lib as L


def real_dtype(prec: str) -> torch.dtype:
    return torch.float64 if prec == "f64" else torch.float32


def _p(t) -> ctypes.c_void_p | None:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class _Workspace:
    """A 256-byte aligned device scratch buffer kept alive by the caller."""

    def __init__(self, nbytes: int, device: torch.device):
        self.nbytes = int(nbytes)
        self.buf = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device) if nbytes > 0 else None
        if self.buf is None:
            self.ptr = None
        else:
            addr = self.buf.data_ptr()
            self.ptr = ctypes.c_void_p((addr + 255) & ~255)


@dataclasses.dataclass
class Hyper:
    kernel: str
    ell: float
    s: float

    def struct(self) -> L.LrHyper:
        return L.LrHyper(L.KERNELS[self.kernel], 0, float(self.ell), float(self.s))


@dataclasses.dataclass
class Omega:
    kind: str
    n: int
    d: int
    signs: torch.Tensor | None = None
    cols: torch.Tensor | None = None
    dense_t: torch.Tensor | None = None
    ld: int = 0

    @staticmethod
    def srht(signs: np.ndarray, cols: np.ndarray, device) -> "Omega":
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        n = int(signs.shape[0])
        L.check(L.lib().lr_check_srht_cols(cols.ctypes.data_as(ctypes.c_void_p), int(cols.shape[0]), n),
                "lr_check_srht_cols")
        return Omega("srht", n, int(cols.shape[0]),
                     signs=torch.from_numpy(np.ascontiguousarray(signs, dtype=np.int8)).to(device),
                     cols=torch.from_numpy(cols).to(device))

    @staticmethod
    def structured(transform: str, signs: np.ndarray, cols: np.ndarray, prec: str, device) -> "Omega":
        """Omega = D T P for T the orthonormal DCT-II ("dct"), the discrete
        Hartley transform ("dht") or Walsh-Hadamard ("wht"), written out on the
        device by lr_structured_omega as a dense transposed Omega (d x ld, ld =
        n rounded up to 64) in the element type of ``prec``."""
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        n, d = int(signs.shape[0]), int(cols.shape[0])
        L.check(L.lib().lr_check_srht_cols(cols.ctypes.data_as(ctypes.c_void_p), d, n), "lr_check_srht_cols")
        ld = (n + 63) // 64 * 64
        dt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "bf16x2": torch.bfloat16}[prec]
        sg = torch.from_numpy(np.ascontiguousarray(signs, dtype=np.int8)).to(device)
        cl = torch.from_numpy(cols).to(device)
        dense = torch.empty((d, ld), dtype=dt, device=device)
        L.check(L.lib().lr_structured_omega(_stream(device), L.TRANSFORMS[transform], n, d, _p(sg), _p(cl),
                                            L.PRECS[prec], _p(dense), ld), "lr_structured_omega")
        return Omega("gauss", n, d, dense_t=dense, ld=ld)

    @staticmethod
    def gauss(omega_t: np.ndarray, prec: str, device) -> "Omega":
        """Omega given transposed (d x n); stored d x ld with ld = n rounded up to 64."""
        d, n = omega_t.shape
        ld = (n + 63) // 64 * 64
        dt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "bf16x2": torch.bfloat16}[prec]
        host = torch.zeros((d, ld), dtype=torch.float32)
        host[:, :n] = torch.from_numpy(np.ascontiguousarray(omega_t, dtype=np.float32))
        if prec == "f64":
            host = host.to(torch.float64)
        return Omega("gauss", n, d, dense_t=host.to(dt).to(device), ld=ld)

    def struct(self) -> L.LrOmega:
        if self.kind == "srht":
            return L.LrOmega(L.LR_OMEGA_SRHT, self.d, self.n, 0, _p(self.signs), _p(self.cols), None)
        return L.LrOmega(L.LR_OMEGA_GAUSS, self.d, self.n, self.ld, None, None, _p(self.dense_t))


def _check_real(t: torch.Tensor, prec: str, name: str) -> None:
    if t.dtype != real_dtype(prec) or not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"{name} must be a contiguous CUDA {real_dtype(prec)} tensor")


def sketch(X: torch.Tensor, hyper: Hyper, omega: Omega, prec: str, nu: float = 0.0, want_y: bool = True,
           want_yprime: bool = False):
    if X.dtype != torch.float32 or not X.is_contiguous():
        raise ValueError("points must be contiguous float32")
    n, D = X.shape
    dev = X.device
    rd = real_dtype(prec)
    Y = torch.empty((n, omega.d), dtype=rd, device=dev) if want_y else None
    Yp = torch.empty((n, omega.d), dtype=rd, device=dev) if want_yprime else None
    lib = L.lib()
    ws = _Workspace(lib.lr_sketch_workspace_bytes(n, D, omega.d, L.PRECS[prec]), dev)
    h, o = hyper.struct(), omega.struct()
    L.check(lib.lr_sketch(_stream(dev), n, D, _p(X), ctypes.byref(h), ctypes.byref(o), float(nu), L.PRECS[prec],
                          _p(Y), _p(Yp), ws.ptr, ws.nbytes), "lr_sketch")
    return Y, Yp


def sketch_grid(X: torch.Tensor, hypers: list, omega: Omega, prec: str, nu: float = 0.0) -> torch.Tensor:
    """Y_g = (K_f(hypers[g]) + nu I) Omega for every g, one lr_sketch_grid call:
    returns a (G, n, d) tensor."""
    if X.dtype != torch.float32 or not X.is_contiguous():
        raise ValueError("points must be contiguous float32")
    n, D = X.shape
    g = len(hypers)
    hs = (L.LrHyper * g)(*[h.struct() for h in hypers])
    Y = torch.empty((g, n, omega.d), dtype=real_dtype(prec), device=X.device)
    lib = L.lib()
    ws = _Workspace(lib.lr_sketch_grid_workspace_bytes(n, D, omega.d, L.PRECS[prec]), X.device)
    o = omega.struct()
    L.check(lib.lr_sketch_grid(_stream(X.device), n, D, _p(X), g, ctypes.cast(hs, ctypes.c_void_p),
                               ctypes.byref(o), float(nu), L.PRECS[prec], _p(Y), ws.ptr, ws.nbytes), "lr_sketch_grid")
    return Y


def loglik_grid(X: torch.Tensor, hypers: list, sigma2s: list, omega: Omega, prec: str, y: torch.Tensor,
                leaf_rows: int, nu: float = 0.0) -> torch.Tensor:
    """Approximate log-likelihoods at a grid of hyperparameters (hypers[g],
    sigma2s[g]): one batched sketch, then the blocked QR, the Woodbury solve
    and lr_loglik per grid point, all on the current stream. Returns a float64
    tensor of G values (NaN where the core is not positive definite)."""
    Ys = sketch_grid(X, hypers, omega, prec, nu=nu)
    out = torch.empty(len(hypers), dtype=torch.float64, device=X.device)
    yc = y.reshape(-1, 1)
    for g in range(len(hypers)):
        Q, R = tsqr(Ys[g], leaf_rows, prec)
        sol = lowrank_solve(Q, R, omega, prec, float(sigma2s[g]), yc, nu=nu)
        out[g:g + 1] = loglik(yc, sol.X, sol.logdet, sol.info, prec)
    return out


def tsqr(Y: torch.Tensor, leaf_rows: int, prec: str):
    _check_real(Y, prec, "Y")
    n, d = Y.shape
    dev = Y.device
    Q = torch.empty_like(Y)
    R = torch.empty((d, d), dtype=torch.float64, device=dev)
    lib = L.lib()
    ws = _Workspace(lib.lr_tsqr_workspace_bytes(n, d, leaf_rows, L.PRECS[prec]), dev)
    L.check(lib.lr_tsqr(_stream(dev), n, d, int(leaf_rows), L.PRECS[prec], _p(Y), _p(Q), _p(R), ws.ptr, ws.nbytes),
            "lr_tsqr")
    return Q, R


@dataclasses.dataclass
class SolveOut:
    X: torch.Tensor | None
    C: torch.Tensor
    L: torch.Tensor
    Flu: torch.Tensor
    piv: torch.Tensor
    logdet: torch.Tensor
    info: torch.Tensor


def tsqr_tree(Y: torch.Tensor, leaf_rows: int, prec: str, group: int = 1, want_q: bool = True):
    """Blocked QR with groups of ``group`` blocks run sequentially (Eq. 5) under
    the binary tree; ``want_q=False`` returns (None, R) without forming Q."""
    _check_real(Y, prec, "Y")
    n, d = Y.shape
    dev = Y.device
    Q = torch.empty_like(Y) if want_q else None
    R = torch.empty((d, d), dtype=torch.float64, device=dev)
    lib = L.lib()
    ws = _Workspace(lib.lr_tsqr_tree_workspace_bytes(n, d, int(leaf_rows), int(group), L.PRECS[prec]), dev)
    L.check(lib.lr_tsqr_tree(_stream(dev), n, d, int(leaf_rows), int(group), L.PRECS[prec], _p(Y), _p(Q), _p(R),
                             ws.ptr, ws.nbytes), "lr_tsqr_tree")
    return Q, R


def lowrank_solve(Q: torch.Tensor, R: torch.Tensor, omega: Omega, prec: str, sigma2: float,
                  A: torch.Tensor | None, nu: float = 0.0) -> SolveOut:
    _check_real(Q, prec, "Q")
    n, d = Q.shape
    dev = Q.device
    m = 0 if A is None else int(A.shape[1])
    if A is not None:
        _check_real(A, prec, "A")
    X = torch.empty_like(A) if A is not None else None
    f64 = dict(dtype=torch.float64, device=dev)
    out = SolveOut(X, torch.empty((d, d), **f64), torch.empty((d, d), **f64), torch.empty((d, d), **f64),
                   torch.empty(d, dtype=torch.int32, device=dev), torch.empty(1, **f64),
                   torch.empty(1, dtype=torch.int32, device=dev))
    lib = L.lib()
    ws = _Workspace(lib.lr_lowrank_solve_workspace_bytes(n, d, m, L.PRECS[prec]), dev)
    o = omega.struct()
    L.check(lib.lr_lowrank_solve(_stream(dev), n, d, m, ctypes.byref(o), L.PRECS[prec], _p(Q), _p(R), float(sigma2),
                                 float(nu), _p(A), _p(X), _p(out.C), _p(out.L), _p(out.Flu), _p(out.piv),
                                 _p(out.logdet), _p(out.info), ws.ptr, ws.nbytes), "lr_lowrank_solve")
    return out


@dataclasses.dataclass
class ProjectionOut:
    X: torch.Tensor | None
    B: torch.Tensor
    L: torch.Tensor
    logdet: torch.Tensor
    info: torch.Tensor


def projection_solve(X: torch.Tensor, hyper: Hyper, Q: torch.Tensor, prec: str, sigma2: float,
                     A: torch.Tensor | None, clip: bool = True) -> ProjectionOut:
    """The projection variant K~ = sigma2 I + Q (Q^T K_f Q) Q^T (B clipped to its
    PSD part with ``clip``) applied to A, through lr_projection_solve."""
    _check_real(Q, prec, "Q")
    if X.dtype != torch.float32 or not X.is_contiguous():
        raise ValueError("points must be contiguous float32")
    n, d = Q.shape
    D = X.shape[1]
    m = 0 if A is None else int(A.shape[1])
    dev = Q.device
    if A is not None:
        _check_real(A, prec, "A")
    out = torch.empty((n, m), dtype=Q.dtype, device=dev) if m > 0 else None
    B = torch.empty((d, d), dtype=torch.float64, device=dev)
    Lf = torch.empty((d, d), dtype=torch.float64, device=dev)
    logdet = torch.empty(1, dtype=torch.float64, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    lib = L.lib()
    ws = _Workspace(lib.lr_projection_solve_workspace_bytes(n, D, d, m, L.PRECS[prec]), dev)
    h = hyper.struct()
    L.check(lib.lr_projection_solve(_stream(dev), n, D, d, _p(X), ctypes.byref(h), L.PRECS[prec], _p(Q),
                                    float(sigma2), 1 if clip else 0, m, _p(A), _p(out), _p(B), _p(Lf), _p(logdet),
                                    _p(info), ws.ptr, ws.nbytes), "lr_projection_solve")
    return ProjectionOut(out, B, Lf, logdet, info)


def psd_part(B: torch.Tensor) -> torch.Tensor:
    """V max(Lambda, 0) V^T of a symmetric float64 d x d device matrix (lr_psd_part)."""
    if B.dtype != torch.float64 or not B.is_contiguous() or B.dim() != 2 or B.shape[0] != B.shape[1]:
        raise ValueError("B must be a contiguous square float64 tensor")
    d = int(B.shape[0])
    out = torch.empty_like(B)
    lib = L.lib()
    ws = _Workspace(lib.lr_psd_part_workspace_bytes(d), B.device)
    L.check(lib.lr_psd_part(_stream(B.device), d, _p(B), _p(out), ws.ptr, ws.nbytes), "lr_psd_part")
    return out


def loglik(y: torch.Tensor, alpha: torch.Tensor, logdet: torch.Tensor, info: torch.Tensor | None,
           prec: str) -> torch.Tensor:
    out = torch.empty(1, dtype=torch.float64, device=y.device)
    L.check(L.lib().lr_loglik(_stream(y.device), int(y.numel()), L.PRECS[prec], _p(y), _p(alpha), _p(logdet),
                              _p(info), _p(out)), "lr_loglik")
    return out


def backward(X: torch.Tensor, hyper: Hyper, omega: Omega, prec: str, fac: SolveOut, Q: torch.Tensor, sigma2: float,
             mode: int, A: torch.Tensor, V: torch.Tensor | None = None, Yprime: torch.Tensor | None = None,
             want_dA: bool = False, R: torch.Tensor | None = None, nu: float = 0.0):
    """Gradient in (log ell, log s, log sigma2). ``A`` is the forward's
    right-hand side (y for mode 0), ``V`` the cotangent Abar (mode 1); with a
    shift ``nu`` the forward's R factor is needed too."""
    n, D = X.shape
    dev = X.device
    _check_real(A, prec, "A")
    if V is not None:
        _check_real(V, prec, "V")
    m = int(A.shape[1]) if A.dim() == 2 else 1
    dtheta = torch.empty(3, dtype=torch.float64, device=dev)
    dA = torch.empty_like(V) if (want_dA and V is not None) else None
    lib = L.lib()
    ws = _Workspace(lib.lr_backward_workspace_bytes(n, D, omega.d, m, L.PRECS[prec]), dev)
    h, o = hyper.struct(), omega.struct()
    L.check(lib.lr_backward(_stream(dev), n, D, _p(X), ctypes.byref(h), ctypes.byref(o), L.PRECS[prec], _p(Q), _p(R),
                            _p(fac.C), _p(fac.L), _p(fac.Flu), _p(fac.piv), float(sigma2), float(nu), int(mode), m,
                            _p(A), _p(V),
                            _p(Yprime), _p(dtheta), _p(dA), ws.ptr, ws.nbytes), "lr_backward")
    return dtheta, dA


@dataclasses.dataclass
class Forward:
    Y: torch.Tensor
    Yprime: torch.Tensor | None
    Q: torch.Tensor
    R: torch.Tensor
    sol: SolveOut


def forward(X: torch.Tensor, hyper: Hyper, omega: Omega, prec: str, sigma2: float, A: torch.Tensor | None,
            leaf_rows: int, nu: float = 0.0, want_yprime: bool = False) -> Forward:
    """Sketch -> blocked QR -> Woodbury solve, all on the current stream."""
    Y, Yp = sketch(X, hyper, omega, prec, nu=nu, want_yprime=want_yprime)
    Q, R = tsqr(Y, leaf_rows, prec)
    sol = lowrank_solve(Q, R, omega, prec, sigma2, A, nu=nu)
    return Forward(Y, Yp, Q, R, sol)


def theta_of(hyper: Hyper, sigma2: float):
    return (math.log(hyper.ell), math.log(hyper.s), math.log(sigma2))
