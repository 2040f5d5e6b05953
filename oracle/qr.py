"""Householder QR and the binary-tree blocked QR of a tall matrix (oracle).

Sec. 3.3, Eq. (1)-(4): split the tall sketch into row blocks K_i, factor each
K_i = Q_i R_i (Eq. 1), stack the R_i and factor pairs of them (Eq. 2), repeat
until one R is left (Eq. 3); the orthogonal factor is the product of the
block-diagonal factors of every level (Eq. 4). Sec. 3.3 lets the block sizes
vary, so any number of leaves is allowed: pairs are formed left to right and
an unpaired last block is carried to the next level unchanged. The last row
block may be shorter than the others but must have at least d rows.

Each small QR is a column-by-column Householder factorisation with the LAPACK
reflector convention: for the column x = (alpha, x2), if x2 = 0 then tau = 0
(H = I); otherwise beta = -sign(alpha) ||x||, sign(0) = +1,
tau = (beta - alpha) / beta, v = (1, x2 / (alpha - beta)), and H = I - tau v v^T
maps x to (beta, 0). Q = H_1 H_2 ... H_d.

The thin Q of the whole matrix is formed top-down: the root's thin factor
applied to I_d gives one d x d block per child; each node passes its block
M down as Q_node [M; 0], and each leaf's block becomes its rows of Q via
Q_leaf [M_leaf; 0]. Finally the signs are fixed so that diag(R) >= 0 (row j of
R and column j of Q are negated together when R_jj < 0), which makes R the
unique triangular factor with non-negative diagonal.

tsqr_grouped runs the other scheme Sec. 3.3 gives, Eq. (5): inside groups of
consecutive blocks the QR goes in sequence, each step factoring the previous
R stacked on the next block; the groups' R factors then meet in the binary
tree (one group of all blocks is the fully sequential scheme; the paper
expects mixtures of the two to be best).

Pins (tests/test_oracle_qr.py): R against numpy.linalg.qr (sign-normalised);
Q R = A and Q^T Q = I to round-off; exact zeros below the diagonal of R; the
tau = 0 case on a zero column; one leaf identical to the plain factorisation;
R independent of the block size (tree shape); the grouped scheme against
LAPACK for every group size, and with group = 1 equal to tsqr.
"""
from __future__ import annotations

import numpy as np


def householder_qr(a: np.ndarray):
    """Unblocked Householder QR of an m x k matrix (m >= k).

    Returns (v, tau, r): v m x k unit lower-trapezoidal reflectors (v[j, j] = 1),
    tau (k,), r k x k upper triangular (exact zeros below the diagonal).
    """
    a = np.array(a, dtype=np.float64, copy=True)
    m, k = a.shape
    if m < k:
        raise ValueError("householder_qr needs at least as many rows as columns")
    tau = np.zeros(k)
    v = np.zeros((m, k))
    for j in range(k):
        alpha = a[j, j]
        x2 = a[j + 1:, j]
        sigma = float(x2 @ x2)
        v[j, j] = 1.0
        if sigma == 0.0:
            tau[j] = 0.0
            continue
        norm = np.sqrt(alpha * alpha + sigma)
        beta = -norm if alpha >= 0.0 else norm
        tau[j] = (beta - alpha) / beta
        v[j + 1:, j] = x2 / (alpha - beta)
        a[j, j] = beta
        a[j + 1:, j] = 0.0
        if j + 1 < k:
            vj = v[j:, j]
            w = vj @ a[j:, j + 1:]
            a[j:, j + 1:] -= tau[j] * np.outer(vj, w)
    r = np.triu(a[:k, :])
    return v, tau, r


def apply_q(v: np.ndarray, tau: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Q B with Q = H_1 ... H_k (H_k is applied first)."""
    out = np.array(b, dtype=np.float64, copy=True)
    k = v.shape[1]
    for j in range(k - 1, -1, -1):
        if tau[j] == 0.0:
            continue
        vj = v[j:, j]
        w = vj @ out[j:, :]
        out[j:, :] -= tau[j] * np.outer(vj, w)
    return out


def thin_q(v: np.ndarray, tau: np.ndarray) -> np.ndarray:
    m, k = v.shape
    e = np.zeros((m, k))
    e[:k, :k] = np.eye(k)
    return apply_q(v, tau, e)


def leaf_bounds(n: int, leaf_rows: int, d: int):
    """Row ranges of the leaves: full blocks of leaf_rows, the last one possibly shorter."""
    if leaf_rows < d:
        raise ValueError("leaf_rows must be >= d")
    bounds = [(r0, min(r0 + leaf_rows, n)) for r0 in range(0, n, leaf_rows)]
    if bounds[-1][1] - bounds[-1][0] < d:
        raise ValueError("last row block has fewer than d rows")
    return bounds


def tsqr(y: np.ndarray, leaf_rows: int, normalize_signs: bool = True):
    """Binary-tree blocked QR of the n x d matrix y. Returns (Q n x d, R d x d)."""
    y = np.asarray(y, dtype=np.float64)
    n, d = y.shape
    bounds = leaf_bounds(n, leaf_rows, d)

    # Eq. (1): independent QR of every row block.
    leaves = [householder_qr(y[r0:r1]) for (r0, r1) in bounds]
    level_r = [lf[2] for lf in leaves]

    # Eq. (2)-(3): pairwise QR of stacked R factors until one is left.
    levels = []  # each level: list of ("pair", (v, tau)) or ("carry", None)
    while len(level_r) > 1:
        nodes, nxt = [], []
        for i in range(0, len(level_r) - 1, 2):
            v, tau, r = householder_qr(np.vstack([level_r[i], level_r[i + 1]]))
            nodes.append(("pair", (v, tau)))
            nxt.append(r)
        if len(level_r) % 2 == 1:
            nodes.append(("carry", None))
            nxt.append(level_r[-1])
        levels.append(nodes)
        level_r = nxt
    r_final = level_r[0].copy()

    # Eq. (4): form the thin Q top-down.
    blocks = [np.eye(d)]
    for nodes in reversed(levels):
        below = []
        for (kind, fac), m in zip(nodes, blocks):
            if kind == "carry":
                below.append(m)
            else:
                v, tau = fac
                stacked = apply_q(v, tau, np.vstack([m, np.zeros((d, d))]))
                below.append(stacked[:d])
                below.append(stacked[d:])
        blocks = below
    q = np.empty((n, d))
    for (r0, r1), (v, tau, _), m in zip(bounds, leaves, blocks):
        rows = r1 - r0
        b = np.zeros((rows, d))
        b[:d] = m
        q[r0:r1] = apply_q(v, tau, b)

    if normalize_signs:
        neg = np.diag(r_final) < 0.0
        r_final[neg, :] *= -1.0
        q[:, neg] *= -1.0
    return q, r_final


def tsqr_grouped(y: np.ndarray, leaf_rows: int, group: int, normalize_signs: bool = True):
    """Blocked QR with the sequential scheme of Eq. (5) inside groups of
    ``group`` consecutive row blocks, and the binary tree of Eq. (2)-(4) over
    the groups' R factors. Inside a group: the QR of the first block, then
    for every further block K_t the QR of [R_{t-1}; K_t]; the group's rows of Q
    follow from [Q_prev R_{t-1}; K_t] = [Q_prev Q_t^top; Q_t^bottom] R_t.
    group = 1 is tsqr itself. Returns (Q n x d, R d x d)."""
    y = np.asarray(y, dtype=np.float64)
    n, d = y.shape
    bounds = leaf_bounds(n, leaf_rows, d)
    if group < 1 or len(bounds) % group != 0:
        raise ValueError("the number of row blocks must be a multiple of group")
    # each group reduced in sequence to (rows of the group, Q_group, R_group)
    groups = []
    for g0 in range(0, len(bounds), group):
        blocks = bounds[g0:g0 + group]
        v, tau, r = householder_qr(y[blocks[0][0]:blocks[0][1]])
        m0 = blocks[0][1] - blocks[0][0]
        qg = apply_q(v, tau, np.vstack([np.eye(d), np.zeros((m0 - d, d))]))
        for (r0, r1) in blocks[1:]:
            v, tau, r = householder_qr(np.vstack([r, y[r0:r1]]))
            qt = apply_q(v, tau, np.vstack([np.eye(d), np.zeros((r1 - r0, d))]))
            qg = np.vstack([qg @ qt[:d], qt[d:]])
        groups.append((blocks[0][0], blocks[-1][1], qg, r))
    # the binary tree over the group R factors (each group a block of rows)
    rows = np.vstack([g[3] for g in groups])
    q_top, r_final = tsqr(rows, d, normalize_signs=False)
    q = np.empty((n, d))
    for k, (r0, r1, qg, _) in enumerate(groups):
        q[r0:r1] = qg @ q_top[k * d:(k + 1) * d]
    if normalize_signs:
        neg = np.diag(r_final) < 0.0
        r_final[neg, :] *= -1.0
        q[:, neg] *= -1.0
    return q, r_final
