"""Write tests/golden/exact_dense_reference.txt: the exact (dense, FP64)
quantities that the randomized low-rank method approximates, at the two
configurations small enough to factor K = K_f + sigma2 I directly:

* the plain FP64 workload (n = 2048, D = 2, SE s = 1, ell = 0.2,
  sigma2 = 1e-4, SRHT d = 64, A 2048 x 4): the exact K^-1 A and log|K|,
  and the method's own error against them (the FP64 oracle's X~ and log|K~|);
* the log-likelihood workload (n = 32768, D = 2, SE s = 1.5, ell = 0.25,
  sigma2 = 1e-2, GP targets): the exact log-likelihood
  -1/2 y^T K^-1 y - 1/2 log|K| and its gradient in (log ell, log s,
  log sigma2), d/dtheta = 1/2 a^T (dK/dtheta) a - 1/2 tr(K^-1 dK/dtheta)
  with a = K^-1 y, from a dense Cholesky factor (the traces column block by
  column block through triangular solves).

Every kernel entry comes from oracle.kernels; the Cholesky factorisation and
the triangular solves are LAPACK's, through torch's CPU linear algebra (the
numpy/scipy LAPACK in this image fails on a 32768 x 32768 factorisation). Nothing here comes from the HIP library. The difference between
these values and the method's is the method's own approximation error (rank
d, Sec. 3.1), which no precision of the GPU path can remove.

Run from the repository root: ``python tests/golden/make_exact_reference.py``
(about ten minutes and 20 GB of memory at n = 32768).
"""
from __future__ import annotations

import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import grad as og, kernels as ok  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_dense_reference.txt")
BLOCK = 2048


def dense_k(x, kind, ell, s, sigma2, deriv=False):
    """K_f + sigma2 I (or dK_f/dlog ell) formed in row blocks, float64."""
    n = x.shape[0]
    k = np.empty((n, n))
    for i0 in range(0, n, BLOCK):
        i1 = min(n, i0 + BLOCK)
        if deriv:
            k[i0:i1] = ok.kernel_matrix_dlogell(kind, x[i0:i1], x, ell, s)
        else:
            k[i0:i1] = ok.kernel_matrix(kind, x[i0:i1], x, ell, s)
    if not deriv:
        k[np.diag_indices(n)] += sigma2
    return k


def chol(k):
    """Lower Cholesky factor of an SPD float64 numpy matrix (torch CPU, LAPACK)."""
    return torch.linalg.cholesky(torch.from_numpy(k))


def chol_solve(lo, b):
    """K^-1 b from the lower Cholesky factor lo of K."""
    bt = torch.from_numpy(np.ascontiguousarray(b.reshape(b.shape[0], -1)))
    return torch.cholesky_solve(bt, lo, upper=False).numpy().reshape(b.shape)


def plain_case(lines):
    w = W.WORKLOADS["C1"]
    x = W.points(w).astype(np.float64)
    a = W.rhs(w).astype(np.float64)
    k = dense_k(x, w.kernel, w.ell, w.s, w.sigma2)
    lo = chol(k)
    x_exact = chol_solve(lo, a)
    ld_exact = 2.0 * float(torch.log(torch.diagonal(lo)).sum())
    signs, cols = W.srht_draw(w)
    om = {"kind": "srht", "signs": signs, "cols": cols}
    fwd = og.forward(W.points(w), w.kernel, w.ell, w.s, w.sigma2, om, W.rhs(w), w.leaf_rows)
    err = float(np.linalg.norm(fwd["X"] - x_exact) / np.linalg.norm(x_exact))
    lines += [
        "# plain FP64 workload: n=2048, SE s=1 ell=0.2, sigma2=1e-4, SRHT d=64, A 2048x4",
        f"c1_x_exact_fro {float(np.linalg.norm(x_exact))!r}",
        f"c1_logdet_exact {ld_exact!r}",
        f"c1_method_x_relerr {err!r}",
        f"c1_method_logdet {float(fwd['logdet'])!r}",
    ]
    for j in range(a.shape[1]):
        lines.append(f"c1_x_exact_col{j}_fro {float(np.linalg.norm(x_exact[:, j]))!r}")


def loglik_case(lines):
    w = W.WORKLOADS["C4"]
    x32 = W.points(w)
    x = x32.astype(np.float64)
    yv = W.gp_targets(w, x32).astype(np.float64)
    n = w.n
    k = dense_k(x, w.kernel, w.ell, w.s, w.sigma2)
    lo = chol(k)
    del k
    alpha = chol_solve(lo, yv)
    ld = 2.0 * float(torch.log(torch.diagonal(lo)).sum())
    ll = -0.5 * float(yv @ alpha) - 0.5 * ld
    # traces tr(K^-1 M) column block by column block: K^-1 E_J by two
    # triangular solves with the Cholesky factor, never the whole inverse
    tr_inv = tr_l = tr_f = 0.0
    q_l = q_f = 0.0
    for j0 in range(0, n, BLOCK):
        j1 = min(n, j0 + BLOCK)
        e = np.zeros((n, j1 - j0))
        e[np.arange(j0, j1), np.arange(j1 - j0)] = 1.0
        kinv = chol_solve(lo, e)                                      # K^-1[:, J]
        del e
        kf = ok.kernel_matrix(w.kernel, x, x[j0:j1], w.ell, w.s)      # K_f[:, J]
        kl = ok.kernel_matrix_dlogell(w.kernel, x, x[j0:j1], w.ell, w.s)
        tr_inv += float(np.trace(kinv[j0:j1]))
        tr_f += float(np.sum(kinv * kf))
        tr_l += float(np.sum(kinv * kl))
        q_f += float(alpha[j0:j1] @ (kf.T @ alpha))
        q_l += float(alpha[j0:j1] @ (kl.T @ alpha))
        del kinv, kf, kl
    del lo
    g = [0.5 * q_l - 0.5 * tr_l,                      # dK/dlog ell = K_l
         q_f - tr_f,                                  # dK/dlog s = 2 K_f
         0.5 * w.sigma2 * float(alpha @ alpha) - 0.5 * w.sigma2 * tr_inv]   # dK/dlog sigma2 = sigma2 I
    lines += [
        "# log-likelihood workload: n=32768, SE s=1.5 ell=0.25, sigma2=1e-2, GP targets (exact dense K)",
        f"c4_logdet_exact {ld!r}",
        f"c4_loglik_exact {ll!r}",
        f"c4_grad_logell_exact {g[0]!r}",
        f"c4_grad_logs_exact {g[1]!r}",
        f"c4_grad_logsigma2_exact {g[2]!r}",
    ]


def main() -> None:
    lines = ["# Exact dense FP64 references (K = K_f + sigma2 I factored directly).",
             "# Written by tests/golden/make_exact_reference.py (oracle.kernels, workloads and LAPACK only)."]
    plain_case(lines)
    loglik_case(lines)
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
