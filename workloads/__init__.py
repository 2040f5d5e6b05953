"""Seeded synthetic inputs for the low-rank covariance-inverse path.

This module only draws random inputs and names the workload presets. It holds
none of the method's arithmetic (no kernel evaluation, no transform, no
factorisation), so both the FP64 oracle and the HIP path can take their
inputs from here without sharing any computation.

Seeds: ``numpy.random.Generator(PCG64([13121869, cfg, stream]))`` with stream
0 = points, 1 = Omega, 2 = right-hand side A, 3 = GP targets, 4 = extra.

Workloads (the paper's synthetic and real-data experiments, Sec. 5, use
uniform points or standardised covariates; here every case is synthetic):

* ``C1``  n=2048, D=2, SE (s=1, ell=0.2, sigma2=1e-4), SRHT d=64, A 2048x4,
  16 leaves of 128 rows, plain FP64 method.
* ``C2``  n=65536, D=3, SE (1, 0.15, 1e-3), SRHT d=256, A 65536x8,
  16 leaves of 4096 rows, FP32 path vs FP64 path.
* ``C3``  n=262144, D=2, Matern-3/2 (1, 0.1, 1e-3), Gaussian Omega N(0,1/d)
  rounded to bf16, d=512, A 262144x16, 64 leaves of 4096 rows, BF16 sketch.
* ``C4``  n=32768, D=2, SE (s=1.5, ell=0.25, sigma2=1e-2), GP targets y,
  SRHT d=256, 8 leaves of 4096 rows, FP32, log-likelihood + gradient.
* ``C5``  n=1048576, D=2, SE (1, 0.05, 1e-3), SRHT d=1024, A n x 16,
  256 leaves of 4096 rows, FP32 forward + fused hyperparameter backward.
* ``C6``  optional stand-in for the paper's 5-covariate real-data study
  (Sec. 5.2): n=131072, D=5 standard-normal covariates, SE, SRHT d=512.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 13121869

STREAM_POINTS = 0
STREAM_OMEGA = 1
STREAM_RHS = 2
STREAM_TARGETS = 3
STREAM_EXTRA = 4


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    cfg: int            # seed index
    n: int
    D: int
    kernel: str         # "se" or "matern32"
    s: float
    ell: float
    sigma2: float
    omega: str          # "srht" or "gauss"
    d: int
    m: int              # right-hand-side columns (1 for the log-likelihood case)
    leaf_rows: int
    prec: str           # "f64", "f32", "bf16"
    points: str = "uniform"   # "uniform" in [0,1)^D or "normal" covariates
    nu: float = 0.0

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


WORKLOADS = {
    "C1": Workload("C1", 1, 2048, 2, "se", 1.0, 0.2, 1e-4, "srht", 64, 4, 128, "f64"),
    "C2": Workload("C2", 2, 65536, 3, "se", 1.0, 0.15, 1e-3, "srht", 256, 8, 4096, "f32"),
    "C3": Workload("C3", 3, 262144, 2, "matern32", 1.0, 0.1, 1e-3, "gauss", 512, 16, 4096, "bf16"),
    "C4": Workload("C4", 4, 32768, 2, "se", 1.5, 0.25, 1e-2, "srht", 256, 1, 4096, "f32"),
    "C5": Workload("C5", 5, 1048576, 2, "se", 1.0, 0.05, 1e-3, "srht", 1024, 16, 4096, "f32"),
    "C6": Workload("C6", 6, 131072, 5, "se", 1.0, 1.0, 1e-2, "srht", 512, 1, 4096, "f32",
                   points="normal"),
}


def rng(cfg: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([SEED_BASE, int(cfg), int(stream)]))


def points(w: Workload, n: int | None = None) -> np.ndarray:
    """n x D float32 points (uniform in [0,1)^D, or standard-normal covariates)."""
    n = w.n if n is None else n
    g = rng(w.cfg, STREAM_POINTS)
    if w.points == "normal":
        return g.standard_normal((n, w.D), dtype=np.float32)
    return g.random((n, w.D), dtype=np.float32)


def srht_draw(w: Workload, n: int | None = None, d: int | None = None):
    """Rademacher signs (int8, +-1) and d distinct sorted column indices (int32)."""
    n = w.n if n is None else n
    d = w.d if d is None else d
    g = rng(w.cfg, STREAM_OMEGA)
    signs = (g.integers(0, 2, n) * 2 - 1).astype(np.int8)
    cols = np.sort(g.choice(n, d, replace=False)).astype(np.int32)
    return signs, cols


def bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest even); return uint16 bits."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_to_f32(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32)


def gauss_omega(w: Workload, n: int | None = None, d: int | None = None,
                round_bf16: bool | None = None) -> np.ndarray:
    """Gaussian Omega, entries N(0, 1/d), stored TRANSPOSED as a d x n float32 array.

    When ``round_bf16`` (default: the workload's precision is bf16) the values are
    rounded to bfloat16 so both sides see exactly the same Omega.
    """
    n = w.n if n is None else n
    d = w.d if d is None else d
    g = rng(w.cfg, STREAM_OMEGA)
    om_t = g.standard_normal((d, n), dtype=np.float32) * np.float32(1.0 / math.sqrt(d))
    if round_bf16 is None:
        round_bf16 = w.prec == "bf16"
    if round_bf16:
        om_t = bf16_to_f32(bf16_bits(om_t))
    return om_t


def rhs(w: Workload, n: int | None = None, m: int | None = None) -> np.ndarray:
    n = w.n if n is None else n
    m = w.m if m is None else m
    return rng(w.cfg, STREAM_RHS).standard_normal((n, m), dtype=np.float32)


def gp_targets(w: Workload, x: np.ndarray, features: int = 4096) -> np.ndarray:
    """Targets drawn from an (approximate) GP with the workload's SE kernel plus noise.

    Random Fourier features: the SE kernel s^2 exp(-r^2/(2 ell^2)) has a Gaussian
    spectral density, so f(x) = s sqrt(2/M) sum_k a_k cos(w_k.x + b_k) with
    w_k ~ N(0, I/ell^2), b_k ~ U[0, 2pi), a_k ~ N(0,1) is a GP draw whose
    covariance converges to the SE kernel as M grows. Noise N(0, sigma2) is added.
    Returns float32 (n,).
    """
    g = rng(w.cfg, STREAM_TARGETS)
    n, D = x.shape
    W = g.standard_normal((D, features)) / w.ell
    b = g.uniform(0.0, 2.0 * math.pi, features)
    a = g.standard_normal(features)
    f = np.zeros(n)
    xd = x.astype(np.float64)
    step = 8192
    for i0 in range(0, n, step):
        f[i0:i0 + step] = np.cos(xd[i0:i0 + step] @ W + b) @ a
    f *= w.s * math.sqrt(2.0 / features)
    y = f + math.sqrt(w.sigma2) * g.standard_normal(n)
    return y.astype(np.float32)


def small(w: Workload, n: int, d: int | None = None, leaf_rows: int | None = None,
          m: int | None = None) -> Workload:
    """A reduced-size variant of a workload (same kernel and hyperparameters)."""
    d = w.d if d is None else d
    leaf_rows = w.leaf_rows if leaf_rows is None else leaf_rows
    m = w.m if m is None else m
    return w.replace(n=n, d=d, leaf_rows=leaf_rows, m=m, name=f"{w.name}-n{n}-d{d}")
