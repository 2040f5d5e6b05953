"""GPU parity of the projection variant (lr_projection_solve: K~ = sigma2 I +
Q (Q^T K_f Q) Q^T with the eig-clip core) and of its PSD part (lr_psd_part),
against the oracle (oracle.lowrank.projection_solve, psd_part).

Bars:
* PSD part: the Newton-Schulz sign iteration against eigh, 1e-11 ||B||_F
  (eigenvalues below ~1e-13 ||B|| may stay unresolved; their clipping moves
  the result by less than themselves).
* B = Q^T K_f Q, stage-wise (the oracle fed the GPU's Q): every entry of the
  second pass K_f Q carries the dense-sketch error (4 sqrt(n) + 16) u of
  sum_j |K_ij| |Q_jk| (float64 or float32 arithmetic), and the exact float64
  sums of Q^T (K_f Q) carry it into B entrywise as that bar times |Q|^T.
  The PSD part is 1-Lipschitz in the Frobenius norm, so the clipped B is held
  to the Frobenius norm of the same bar.
* X and log|K~|, stage-wise (the oracle's Cholesky, apply and log-det fed the
  GPU's Q and B): 1e-10 relative in float64; for float32 X, 1e-5 of max |X|
  (the float32 apply), log|K~| 1e-10 (float64 core).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import kernels, lowrank as olr, qr as oqr, sketch as osk

from conftest import read_golden
from gpu_common import U32, U64, api, device, hyper, note, omega_pair, rel_max, to_dev, torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d", [16, 100, 256, 512])
def test_psd_part_against_eigh(d):
    dev = device()
    a = api()
    rng = np.random.default_rng(d)
    v, _ = np.linalg.qr(rng.standard_normal((d, d)))
    lam = rng.standard_normal(d) * np.logspace(0, -8, d)       # magnitudes down to 1e-8
    lam[:3] = [1e-6, -1e-6, -1e-15]
    b = (v * lam) @ v.T
    b = 0.5 * (b + b.T)
    note(f"psd part d={d}")
    bp = a.psd_part(to_dev(b, torch.float64, dev))
    torch.cuda.synchronize()
    ref = olr.psd_part(b)
    err = np.abs(bp.cpu().numpy() - ref).max()
    note(f"  max |B+ - B+_ref| {err:.2e} (||B||_F {np.linalg.norm(b):.2e})")
    assert err <= 1e-11 * np.linalg.norm(b)


def _b_bar(x, w, q, u):
    """Entrywise bar on B = Q^T K_f Q from the second pass's rounding."""
    kabs = np.abs(kernels.kernel_matrix(w.kernel, x, x, w.ell, w.s))
    sk = kabs @ np.abs(q)
    return (4 * math.sqrt(w.n) + 16) * u * (np.abs(q).T @ sk)


def _stagewise(r, q, sigma2, a_mat):
    """The oracle's Cholesky, log-det and apply fed the GPU's Q and B."""
    b = r.B.cpu().numpy()
    lo, info = olr.cholesky_info(b + sigma2 * np.eye(b.shape[0]))
    assert info == 0
    return olr.apply(q, lo, a_mat, sigma2), olr.logdet(lo, q.shape[0], sigma2)


@pytest.mark.parametrize("prec,clip", [("f64", True), ("f64", False), ("f32", True), ("bf16", True)])
def test_projection_solve_stagewise(prec, clip):
    dev = device()
    a = api()
    w = W.small(W.WORKLOADS["C3"], 3000, d=64, leaf_rows=1000, m=3)
    x = W.points(w)
    xd = x.astype(np.float64)
    A = W.rhs(w)
    om_np, om = omega_pair(w, prec, dev)
    rp = "f64" if prec == "f64" else "f32"
    dt = torch.float64 if rp == "f64" else torch.float32
    X = to_dev(x, torch.float32, dev)
    note(f"projection solve {prec} clip={clip} n={w.n} d={w.d}")
    Y, _ = a.sketch(X, hyper(w), om, prec)
    Q, R = a.tsqr(Y, w.leaf_rows, prec)
    r = a.projection_solve(X, hyper(w), Q, prec, w.sigma2, to_dev(A, dt, dev), clip=clip)
    torch.cuda.synchronize()
    assert int(r.info.item()) == 0
    q = Q.double().cpu().numpy()
    kq = kernels.kernel_matrix(w.kernel, xd, xd, w.ell, w.s) @ q
    b_ref = q.T @ kq
    b_ref = 0.5 * (b_ref + b_ref.T)
    u = U64 if rp == "f64" else U32
    bar = _b_bar(xd, w, q, u)
    b = r.B.cpu().numpy()
    if clip:
        eb = np.linalg.norm(b - olr.psd_part(b_ref))
        note(f"  ||B+ - psd(B_ref)||_F {eb:.2e} (bar {np.linalg.norm(bar):.2e})")
        assert eb <= np.linalg.norm(bar) + 1e-11 * np.linalg.norm(b_ref)
    else:
        eb = (np.abs(b - b_ref) / bar).max()
        note(f"  max |B - B_ref| / bar {eb:.2e}")
        assert eb <= 1.0
    x_st, ld_st = _stagewise(r, q, w.sigma2, A)
    ex = rel_max(r.X.double().cpu().numpy(), x_st)
    el = abs(r.logdet.item() - ld_st) / abs(ld_st)
    note(f"  stage-wise X rel {ex:.2e} logdet rel {el:.2e}")
    assert el <= 1e-10
    assert ex <= (1e-10 if rp == "f64" else 1e-5)
    if prec == "f64":
        # end to end against the oracle's own sketch, tree QR and projection
        y_o = osk.sketch(x, w.kernel, w.ell, w.s, om_np)
        q_o, _ = oqr.tsqr(y_o, w.leaf_rows)
        kq_o = kernels.kernel_matrix(w.kernel, xd, xd, w.ell, w.s) @ q_o
        ref = olr.projection_solve(q_o, kq_o, w.sigma2, A, clip=clip)
        e2 = rel_max(r.X.cpu().numpy(), ref["X"])
        l2 = abs(r.logdet.item() - ref["logdet"]) / abs(ref["logdet"])
        note(f"  end to end X rel {e2:.2e} logdet rel {l2:.2e}")
        assert e2 <= 1e-10 and l2 <= 1e-10


def test_c4_full_fp32_projection_without_shift():
    """The full log-likelihood workload in FP32 with no shift: the Nystrom core
    breaks down here (test_gpu_backward), the projection core does not. B
    stage-wise against the oracle fed the GPU's Q (the PSD part within the
    Frobenius norm of the second pass's bar), the log-likelihood stage-wise,
    and its distance from the exact dense value reported (targets: the seeded
    random-Fourier-feature GP draw of workloads.gp_targets)."""
    dev = device()
    a = api()
    w = W.WORKLOADS["C4"]
    x = W.points(w)
    xd = x.astype(np.float64)
    yv = W.gp_targets(w, x)
    om_np, om = omega_pair(w, "f32", dev)
    X = to_dev(x, torch.float32, dev)
    note(f"C4 full fp32 projection n={w.n} d={w.d} nu=0")
    Y, _ = a.sketch(X, hyper(w), om, "f32")
    Q, R = a.tsqr(Y, w.leaf_rows, "f32")
    yd = to_dev(yv.reshape(-1, 1), torch.float32, dev)
    r = a.projection_solve(X, hyper(w), Q, "f32", w.sigma2, yd, clip=True)
    ll = a.loglik(yd, r.X, r.logdet, r.info, "f32").item()
    torch.cuda.synchronize()
    assert int(r.info.item()) == 0
    q = Q.double().cpu().numpy()
    kq = osk.sketch(x, w.kernel, w.ell, w.s, {"kind": "gauss", "omega_t": q.T})
    b_ref = q.T @ kq
    b_ref = 0.5 * (b_ref + b_ref.T)
    kabs_q = osk.sketch(x, w.kernel, w.ell, w.s, {"kind": "gauss", "omega_t": np.abs(q).T})  # |K_f| |Q| (K_f >= 0)
    bar = (4 * math.sqrt(w.n) + 16) * U32 * (np.abs(q).T @ kabs_q)
    eb = np.linalg.norm(r.B.cpu().numpy() - olr.psd_part(b_ref))
    x_st, ld_st = _stagewise(r, q, w.sigma2, yv.reshape(-1, 1))
    ll_st = olr.loglik(yv, x_st[:, 0], ld_st)
    ex = {k: float(v) for k, v in read_golden("exact_dense_reference.txt")}
    note(f"  ||B+ - psd(B_ref)||_F {eb:.2e} (bar {np.linalg.norm(bar):.2e}); loglik {ll:.8e} stage-wise "
         f"{ll_st:.8e}; against the exact dense log-likelihood {ll - ex['c4_loglik_exact']:+.4e}")
    assert eb <= np.linalg.norm(bar)
    assert abs(ll - ll_st) <= 1e-6 * abs(ll_st)
