"""Walsh-Hadamard transform and the structured random matrix (oracle).

Def. 1 (Sec. 3.2): Omega = c R T P with R an n x n diagonal of independent
Rademacher signs, T an orthogonal fast transform, P an n x d column subset of
the identity, and c chosen so the columns of Omega are orthonormal. Here T is
the Walsh-Hadamard matrix H_n of Sec. 3.2, built by the Sylvester recursion
H_n = [[H_{n/2}, H_{n/2}], [H_{n/2}, -H_{n/2}]], H_2 = [[1, 1], [1, -1]], so n
must be a power of two. Since H_n H_n = n I, c = n^(-1/2) makes Omega^T Omega =
I_d exactly. Entry form: Omega[j, k] = c D_j H[j, P_k], with
H[j, p] = (-1)^popcount(j & p) in the recursion's natural order (0-based).

Pins (tests/test_oracle_srht.py): the recursion against scipy.linalg.hadamard;
the fast transform against the explicit matrix; H(Hx) = n x; Omega^T Omega = I;
the row-transform form of K Omega against the explicit dense product.
"""
from __future__ import annotations

import numpy as np


def is_pow2(n: int) -> bool:
    return n >= 1 and (n & (n - 1)) == 0


def hadamard_sylvester(n: int) -> np.ndarray:
    """H_n by the Sylvester recursion (n a power of 2, n >= 1)."""
    if not is_pow2(n):
        raise ValueError("Walsh-Hadamard order must be a power of two")
    h = np.ones((1, 1))
    while h.shape[0] < n:
        h = np.block([[h, h], [h, -h]])
    return h


def fwht(v: np.ndarray, axis: int = -1) -> np.ndarray:
    """H_n v along ``axis`` by log2(n) butterfly passes (a, b) -> (a + b, a - b).

    Each pass h = 1, 2, 4, ... combines entries whose indices differ in bit h,
    which is the Sylvester recursion applied from the innermost level out.
    """
    a = np.moveaxis(np.array(v, dtype=np.float64, copy=True), axis, -1)
    n = a.shape[-1]
    if not is_pow2(n):
        raise ValueError("Walsh-Hadamard length must be a power of two")
    h = 1
    while h < n:
        a = a.reshape(a.shape[:-1] + (n // (2 * h), 2, h))
        top = a[..., 0, :] + a[..., 1, :]
        bot = a[..., 0, :] - a[..., 1, :]
        a = np.stack([top, bot], axis=-2).reshape(a.shape[:-3] + (n,))
        h *= 2
    return np.moveaxis(a, -1, axis)


def srht_scale(n: int) -> float:
    return 1.0 / np.sqrt(float(n))


def srht_dense(signs: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Explicit n x d Omega = c diag(D) H_n[:, P] (small n only)."""
    n = signs.shape[0]
    h = hadamard_sylvester(n)
    return srht_scale(n) * (signs.astype(np.float64)[:, None] * h[:, np.asarray(cols)])


def right_apply(m: np.ndarray, signs: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """M Omega for an r x n matrix M: each row becomes c (H (D o m_i))[P]  (H symmetric)."""
    n = signs.shape[0]
    t = fwht(np.asarray(m, dtype=np.float64) * signs.astype(np.float64)[None, :], axis=1)
    return srht_scale(n) * t[:, np.asarray(cols)]


def left_apply_t(q: np.ndarray, signs: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Omega^T Q for an n x r matrix Q: c P^T H D Q, via the transform of each column."""
    n = signs.shape[0]
    t = fwht(signs.astype(np.float64)[:, None] * np.asarray(q, dtype=np.float64), axis=0)
    return srht_scale(n) * t[np.asarray(cols), :]


def entries(signs: np.ndarray, cols: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """Omega[rows, :] from the entry formula c D_j (-1)^popcount(j & P_k)."""
    n = signs.shape[0]
    rows = np.asarray(rows, dtype=np.int64)
    p = np.asarray(cols, dtype=np.int64)
    andv = rows[:, None] & p[None, :]
    parity = np.zeros(andv.shape, dtype=np.int64)
    x = andv.copy()
    while np.any(x):
        parity ^= x & 1
        x >>= 1
    sign_h = 1.0 - 2.0 * parity
    return srht_scale(n) * signs.astype(np.float64)[rows][:, None] * sign_h
