"""Woodbury-form approximate inverse, log-determinant and log-likelihood (oracle).

The paper's target is K^{-1} A for a huge SPD K (Sec. 1) through a QR of the
sketch K Omega (Sec. 3.1, Sec. 3.3) and the projection of K onto its column
space (Sec. 3.1; proof of Thm 5), but it never writes the final formula. The
reading used here (see the design notes) is the projected-process / Nystrom
approximation of the signal covariance from the sketch, with the nugget added
back exactly:

    Y = (K_f + nu I) Omega = Q R,   W = Omega^T Y,
    K_tilde = sigma2 I + Y W^{-1} Y^T - nu Q Q^T.

Because Y W^{-1} Y^T = Q R (F R)^{-1} R^T Q^T = Q F^{-1} R^T Q^T with
F = Omega^T Q, the ill-conditioned W is never inverted:

    C = sym(F^{-1} R^T)   (LU of F with partial pivoting; sym(M) = (M + M^T)/2)
    S = C + (sigma2 - nu) I = L L^T        (Cholesky; info = k if the k-th pivot <= 0)
    K_tilde^{-1} A = sigma2^{-1} (A - Q Z) + Q S^{-1} Z,   Z = Q^T A
    log|K_tilde|  = (n - d) log sigma2 + 2 sum_j log L_jj
    loglik        = -1/2 y^T K_tilde^{-1} y - 1/2 log|K_tilde|   (no -n/2 log 2 pi)

Projection variant (the symmetric form of the object Q Q^T K that Sec. 3.1
bounds in Thm 5, with the further products Sec. 3.3 expects after the QR):

    B = Q^T K_f Q,  optionally replaced by its positive semidefinite part
        V max(Lambda, 0) V^T (B = V Lambda V^T; the eig-clip core),
    K_tilde = sigma2 I + Q B Q^T,  S = B + sigma2 I = L L^T,

with the same apply and log-determinant. B is positive semidefinite in exact
arithmetic for any orthonormal Q; the clip removes what rounding leaves.

Pins (tests/test_oracle_lowrank.py): the dense definition (sigma2 I + Y W^{-1}
Y^T - nu P_Y)^{-1} A and slogdet on small n; exact recovery of K^{-1} A when
K_f has rank <= d; exact recovery when d = n (Omega orthogonal); K_f = 0 gives
A / sigma2; invariance under Omega -> Omega T for orthogonal T; the Cholesky
info convention on an indefinite S. Projection: the dense definition
(sigma2 I + Q Q^T K_f Q Q^T)^{-1} A; exact recovery when range(Q) holds the
range of a low-rank K_f; the PSD part against the nearest positive
semidefinite matrix in the Frobenius norm (its distance is the norm of the
negative eigenvalues), idempotence, and a PSD input left unchanged.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .sketch import omega_t_apply


def cholesky_info(s: np.ndarray):
    """Cholesky S = L L^T column by column. Returns (L, info), info = 0 or the
    1-based index of the first non-positive pivot (L is then partial)."""
    s = np.asarray(s, dtype=np.float64)
    d = s.shape[0]
    lo = np.zeros((d, d))
    for j in range(d):
        ajj = s[j, j] - lo[j, :j] @ lo[j, :j]
        if not (ajj > 0.0):
            return lo, j + 1
        ljj = np.sqrt(ajj)
        lo[j, j] = ljj
        if j + 1 < d:
            lo[j + 1:, j] = (s[j + 1:, j] - lo[j + 1:, :j] @ lo[j, :j]) / ljj
    return lo, 0


def core(q: np.ndarray, r: np.ndarray, omega: dict, sigma2: float, nu: float = 0.0):
    """F = Omega^T Q, C = sym(F^{-1} R^T), S = C + (sigma2 - nu) I, S = L L^T.

    Returns a dict with F, lu (scipy LU factors), C, S, L, info.
    """
    f = omega_t_apply(omega, q)
    lu = sla.lu_factor(f, check_finite=False)
    c = sla.lu_solve(lu, np.asarray(r, dtype=np.float64).T, check_finite=False)
    c = 0.5 * (c + c.T)
    d = c.shape[0]
    s = c + (sigma2 - nu) * np.eye(d)
    lo, info = cholesky_info(s)
    return {"F": f, "lu": lu, "C": c, "S": s, "L": lo, "info": info}


def s_solve(lo: np.ndarray, z: np.ndarray) -> np.ndarray:
    """S^{-1} Z with S = L L^T (forward then backward substitution)."""
    t = sla.solve_triangular(lo, z, lower=True, check_finite=False)
    return sla.solve_triangular(lo.T, t, lower=False, check_finite=False)


def apply(q: np.ndarray, lo: np.ndarray, a: np.ndarray, sigma2: float) -> np.ndarray:
    """K_tilde^{-1} A = sigma2^{-1} (A - Q Z) + Q S^{-1} Z, Z = Q^T A."""
    q = np.asarray(q, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    z = q.T @ a
    w = s_solve(lo, z)
    return (a - q @ z) / sigma2 + q @ w


def logdet(lo: np.ndarray, n: int, sigma2: float) -> float:
    d = lo.shape[0]
    return (n - d) * np.log(sigma2) + 2.0 * float(np.sum(np.log(np.diag(lo))))


def loglik(y: np.ndarray, alpha: np.ndarray, ld: float) -> float:
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    return -0.5 * float(y @ np.asarray(alpha).reshape(-1)) - 0.5 * ld


def solve(q, r, omega, sigma2, a, nu=0.0):
    """Whole Woodbury stage: returns dict with X, logdet, and the core factors."""
    c = core(q, r, omega, sigma2, nu)
    if c["info"] != 0:
        c["X"] = None
        c["logdet"] = np.nan
        return c
    c["X"] = apply(q, c["L"], a, sigma2)
    c["logdet"] = logdet(c["L"], np.asarray(q).shape[0], sigma2)
    return c


# ---------------------------------------------------------------- dense definitions

def k_tilde_dense(y: np.ndarray, omega_dense: np.ndarray, sigma2: float,
                  nu: float = 0.0) -> np.ndarray:
    """sigma2 I + Y W^{-1} Y^T - nu P_Y, W = Omega^T Y, P_Y the projector onto range(Y)."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    w = omega_dense.T @ y
    kt = sigma2 * np.eye(n) + y @ np.linalg.solve(w, y.T)
    if nu != 0.0:
        kt -= nu * (y @ np.linalg.solve(y.T @ y, y.T))
    return 0.5 * (kt + kt.T)


def solve_dense(y, omega_dense, sigma2, a, nu=0.0):
    kt = k_tilde_dense(y, omega_dense, sigma2, nu)
    x = np.linalg.solve(kt, np.asarray(a, dtype=np.float64))
    sign, ld = np.linalg.slogdet(kt)
    return x, ld, sign


# ---------------------------------------------------------------- projection variant

def psd_part(b: np.ndarray) -> np.ndarray:
    """V max(Lambda, 0) V^T for symmetric b = V Lambda V^T (eigh)."""
    b = 0.5 * (np.asarray(b, dtype=np.float64) + np.asarray(b, dtype=np.float64).T)
    lam, v = np.linalg.eigh(b)
    return (v * np.maximum(lam, 0.0)) @ v.T


def projection_core(q: np.ndarray, kq: np.ndarray, sigma2: float, clip: bool = True):
    """B = sym(Q^T (K_f Q)) from the second pass kq = K_f Q, optionally clipped
    to its PSD part; S = B + sigma2 I = L L^T. Returns dict(B, L, info)."""
    q = np.asarray(q, dtype=np.float64)
    b = q.T @ np.asarray(kq, dtype=np.float64)
    b = 0.5 * (b + b.T)
    if clip:
        b = psd_part(b)
    lo, info = cholesky_info(b + sigma2 * np.eye(b.shape[0]))
    return {"B": b, "L": lo, "info": info}


def projection_solve(q, kq, sigma2, a, clip=True):
    """The projection variant's K_tilde^{-1} A and log|K_tilde| (dict with X,
    logdet, B, L, info)."""
    c = projection_core(q, kq, sigma2, clip)
    if c["info"] != 0:
        c["X"], c["logdet"] = None, np.nan
        return c
    c["X"] = apply(q, c["L"], a, sigma2)
    c["logdet"] = logdet(c["L"], np.asarray(q).shape[0], sigma2)
    return c
