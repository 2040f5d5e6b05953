"""The sketch Y = (K_f + nu I) Omega (oracle).

Sec. 3.1: the column space of K is approximated by that of K Omega, Omega n x d
random with d << n. Sec. 3.2: with a structured Omega the product needs only a
fast transform per row of K. K_f[i, j] = k(x_i, x_j) is the signal covariance;
nu shifts the sketched matrix (nu = 0 sketches K_f itself, nu = sigma2 sketches
the full K = K_f + sigma2 I). Row i of Y depends only on x_i and all points, so
any subset of rows can be computed on its own (used for sampled parity).

Omega is described by a small dict:
  {"kind": "srht", "signs": int8[n], "cols": int32[d]}
  {"kind": "dct" or "dht", "signs": int8[n], "cols": int32[d]}  (transforms.py)
  {"kind": "gauss", "omega_t": float[d, n]}   (Omega stored transposed)

Precision model (for the bf16 matrix-core paths): ``k_round="bf16"`` rounds each
K_f entry to bfloat16 (round to nearest even) before the product;
``k_round="bf16x2"`` replaces each entry k by k_hi + k_lo with k_hi = bf16(k)
and k_lo = bf16(k - k_hi) (a two-term split that keeps about 16 bits, the
product of both terms with Omega summed). Omega is already bf16-valued in
that workload. Default: no rounding.

Pins (tests/test_oracle_sketch.py): explicit dense K_f @ Omega on small n for
both Omega kinds; the row-sampled form against the full product; linearity in
Omega; nu shift against the explicit (K_f + nu I) Omega.
"""
from __future__ import annotations

import numpy as np

from . import kernels, srht, transforms


def omega_dense(omega: dict, n: int) -> np.ndarray:
    """Explicit n x d Omega (small n only)."""
    if omega["kind"] == "srht":
        return srht.srht_dense(omega["signs"], omega["cols"])
    if omega["kind"] in transforms.KINDS:
        return transforms.omega_dense(omega["kind"], omega["signs"], omega["cols"])
    return np.asarray(omega["omega_t"], dtype=np.float64).T.copy()


def omega_rows(omega: dict, rows: np.ndarray) -> np.ndarray:
    """Omega[rows, :] as float64."""
    rows = np.asarray(rows, dtype=np.int64)
    if omega["kind"] == "srht":
        return srht.entries(omega["signs"], omega["cols"], rows)
    if omega["kind"] in transforms.KINDS:
        return transforms.omega_entries(omega["kind"], omega["signs"], omega["cols"], rows)
    return np.asarray(omega["omega_t"], dtype=np.float64)[:, rows].T.copy()


def omega_d(omega: dict) -> int:
    if omega["kind"] == "srht" or omega["kind"] in transforms.KINDS:
        return int(np.asarray(omega["cols"]).shape[0])
    return int(np.asarray(omega["omega_t"]).shape[0])


def round_to_bf16(a: np.ndarray) -> np.ndarray:
    """Round float64 values to 8 significant bits, ties to even (bfloat16 grid)."""
    mant, expo = np.frexp(np.asarray(a, dtype=np.float64))
    return np.ldexp(np.rint(mant * 256.0), expo - 8)


def round_to_bf16x2(a: np.ndarray) -> np.ndarray:
    """k_hi + k_lo with k_hi = bf16(k), k_lo = bf16(k - k_hi), summed in float64."""
    a = np.asarray(a, dtype=np.float64)
    hi = round_to_bf16(a)
    return hi + round_to_bf16(a - hi)


def _right_apply(kblock: np.ndarray, omega: dict) -> np.ndarray:
    if omega["kind"] == "srht":
        return srht.right_apply(kblock, omega["signs"], omega["cols"])
    if omega["kind"] in transforms.KINDS:
        return transforms.right_apply(kblock, omega["kind"], omega["signs"], omega["cols"])
    return kblock @ np.asarray(omega["omega_t"], dtype=np.float64).T


def sketch_rows(x: np.ndarray, rows: np.ndarray, kind: str, ell: float, s: float,
                omega: dict, nu: float = 0.0, deriv: bool = False,
                k_round: str | None = None, block: int = 256) -> np.ndarray:
    """Y[rows, :] = K_f[rows, :] Omega + nu Omega[rows, :].

    With ``deriv`` the derivative sketch (dK_f/dlog ell) Omega is returned instead
    (no nu term: the shift does not depend on ell).
    """
    rows = np.asarray(rows, dtype=np.int64)
    x64 = np.asarray(x, dtype=np.float64)
    d = omega_d(omega)
    out = np.empty((rows.shape[0], d))
    for b0 in range(0, rows.shape[0], block):
        rb = rows[b0:b0 + block]
        if deriv:
            kb = kernels.kernel_matrix_dlogell(kind, x64[rb], x64, ell, s)
        else:
            kb = kernels.kernel_matrix(kind, x64[rb], x64, ell, s)
        if k_round == "bf16":
            kb = round_to_bf16(kb)
        elif k_round == "bf16x2":
            kb = round_to_bf16x2(kb)
        out[b0:b0 + block] = _right_apply(kb, omega)
    if nu != 0.0 and not deriv:
        out += nu * omega_rows(omega, rows)
    return out


def sketch(x: np.ndarray, kind: str, ell: float, s: float, omega: dict, nu: float = 0.0,
           deriv: bool = False, k_round: str | None = None) -> np.ndarray:
    """Full Y = (K_f + nu I) Omega (n x d)."""
    n = np.asarray(x).shape[0]
    return sketch_rows(x, np.arange(n), kind, ell, s, omega, nu, deriv, k_round)


def omega_t_apply(omega: dict, q: np.ndarray) -> np.ndarray:
    """Omega^T Q (d x r)."""
    if omega["kind"] == "srht":
        return srht.left_apply_t(q, omega["signs"], omega["cols"])
    if omega["kind"] in transforms.KINDS:
        return transforms.left_apply_t(q, omega["kind"], omega["signs"], omega["cols"])
    return np.asarray(omega["omega_t"], dtype=np.float64) @ np.asarray(q, dtype=np.float64)
