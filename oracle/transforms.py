"""Structured random matrices built on the discrete cosine and Hartley
transforms (oracle).

Sec. 3.2 allows any fast orthogonal transform T in Omega = R T P (Def. 1) and
names the discrete cosine and the discrete Hartley transforms as the real
alternatives to Walsh-Hadamard that exist for every n (no power-of-two
restriction); the experiments of Sec. 5 use both (Table 3: HP and HC). The
paper does not fix their normalisation. Reading: the orthonormal forms,

  DCT-II:  T[j, p] = a_p cos(pi (2j + 1) p / (2n)),  a_0 = n^-1/2, a_p = (2/n)^1/2
  DHT:     T[j, p] = n^-1/2 cas(2 pi j p / n),       cas t = cos t + sin t

so T is orthogonal, Omega[j, k] = D_j T[j, P_k] has orthonormal columns
(Omega^T Omega = I_d exactly, c = 1) and K~ is invariant to the choice
exactly as for Walsh-Hadamard. D is the Rademacher diagonal and P the d
columns (drawn without replacement, sorted), as in srht.py.

Entries come from the formulas above with the angle reduced exactly in
integers to the first octant before the float64 cosine or sine (the Hartley
entry as sqrt(2) cos(t - pi/4)), so exact zeros stay zero.
The products K Omega and Omega^T Q use fast transforms (scipy.fft) along the
transform axis, then pick the columns P.

Pins (tests/test_oracle_transforms.py): the entry formulas against
scipy.fft.dct / scipy.fft.fft of the identity; Omega^T Omega = I; the DHT
matrix is its own inverse; the DCT of a constant vector is a multiple of e_0;
the fast right and left applies against the explicit dense matrix.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

KINDS = ("dct", "dht")


def cos_pi_ratio(k: np.ndarray, big_n: int) -> np.ndarray:
    """cos(pi k / N) for integers k, with the quadrant reduced in integers
    (cos(-a) = cos a, cos(pi - a) = -cos a, cos a = sin(pi/2 - a)), so the
    float64 cosine or sine only sees an angle in [0, pi/4] and zeros come out
    exactly zero."""
    k = np.mod(np.asarray(k, dtype=np.int64), 2 * big_n)   # [0, 2N)
    k = np.where(k > big_n, 2 * big_n - k, k)               # [0, N]
    sign = np.where(2 * k > big_n, -1.0, 1.0)
    k = np.where(2 * k > big_n, big_n - k, k)               # [0, N/2]
    use_sin = 4 * k > big_n
    return sign * np.where(use_sin, np.sin(np.pi * (big_n - 2 * k) / (2.0 * big_n)),
                           np.cos(np.pi * k / float(big_n)))


def transform_entries(kind: str, n: int, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """T[rows, cols] (float64) from the closed forms, angles reduced in integers."""
    j = np.asarray(rows, dtype=np.int64)[:, None]
    p = np.asarray(cols, dtype=np.int64)[None, :]
    if kind == "dct":
        a = np.where(p == 0, np.sqrt(1.0 / n), np.sqrt(2.0 / n))
        return a * cos_pi_ratio((2 * j + 1) * p, 2 * n)          # cos(pi (2j+1) p / (2n))
    if kind == "dht":
        # cas t = cos t + sin t = sqrt(2) cos(t - pi/4), t = 2 pi m / n
        m = (j * p) % n
        return np.sqrt(2.0) * cos_pi_ratio(8 * m - n, 4 * n) / np.sqrt(n)
    raise ValueError(f"unknown transform {kind!r}")


def omega_entries(kind: str, signs: np.ndarray, cols: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """Omega[rows, :] = D[rows] T[rows, P] (len(rows) x d)."""
    rows = np.asarray(rows, dtype=np.int64)
    n = np.asarray(signs).shape[0]
    d_j = np.asarray(signs, dtype=np.float64)[rows]
    return d_j[:, None] * transform_entries(kind, n, rows, cols)


def omega_dense(kind: str, signs: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Explicit n x d Omega (small n only)."""
    n = np.asarray(signs).shape[0]
    return omega_entries(kind, signs, cols, np.arange(n))


def _transform_rows(m: np.ndarray, kind: str) -> np.ndarray:
    """(T^T v) for every row v of m: DCT-II or DHT along axis 1, orthonormal."""
    if kind == "dct":
        return scipy.fft.dct(m, type=2, norm="ortho", axis=1)
    if kind == "dht":
        f = scipy.fft.fft(m, axis=1)
        return (f.real - f.imag) / np.sqrt(m.shape[1])
    raise ValueError(f"unknown transform {kind!r}")


def right_apply(m: np.ndarray, kind: str, signs: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """M Omega for M (r x n): row i of the result is (T^T (D o m_i))[P]."""
    m = np.asarray(m, dtype=np.float64)
    t = _transform_rows(m * np.asarray(signs, dtype=np.float64)[None, :], kind)
    return t[:, np.asarray(cols, dtype=np.int64)]


def left_apply_t(q: np.ndarray, kind: str, signs: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Omega^T Q (d x r) = (M Omega)^T with M = Q^T."""
    return right_apply(np.asarray(q, dtype=np.float64).T, kind, signs, cols).T
