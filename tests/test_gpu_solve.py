"""GPU parity of the whole forward (sketch -> tsqr -> lowrank_solve) and of
lr_lowrank_solve on its own, against the oracle.

FP64 path: X and log|K~| within 1e-10 relative (the oracle and the GPU run the
same algorithm in float64; differences are rounding order amplified by the
conditioning of the d x d core). FP32 / BF16 paths are compared with the FP64
oracle and with the oracle's precision model of that path: the GPU's own
sketch (a stage input: its float32 values, and for BF16 its bf16-rounded
float32 kernel entries, whose rounding may fall on either side of a bf16
midpoint from the oracle's float64 evaluation), a float32 Householder QR
(LAPACK, gpu_common.qr_fp32), then the float64 core and solve. The model's
distance from the exact oracle measures how strongly the float64 method
reacts to that rounding; the GPU's float32 QR differs from LAPACK's in detail
but not in size, so the bars are a fixed floor plus 4x that distance.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import grad as og, lowrank as olr, sketch as osk

from gpu_common import api, device, hyper, note, omega_pair, qr_fp32, rel_max, to_dev, torch

pytestmark = pytest.mark.gpu


def _forward(w, prec, dev, nu=0.0, m=None):
    a = api()
    x = W.points(w)
    A = W.rhs(w, m=m)
    om_np, om = omega_pair(w, prec, dev)
    rp = "f32" if prec in ("bf16", "bf16x2") else prec
    dt = torch.float64 if rp == "f64" else torch.float32
    note(f"forward {w.name} n={w.n} d={w.d} m={A.shape[1]} prec={prec} nu={nu}")
    Y, _ = a.sketch(to_dev(x, torch.float32, dev), hyper(w), om, prec, nu=nu)
    Q, R = a.tsqr(Y, w.leaf_rows, rp)
    sol = a.lowrank_solve(Q, R, om, prec, w.sigma2, to_dev(A, dt, dev), nu=nu)
    torch.cuda.synchronize()
    return x, A, om_np, om, Y, Q, R, sol


def test_c1_fp64_end_to_end():
    dev = device()
    w = W.WORKLOADS["C1"]
    x, A, om_np, _, Y, Q, R, sol = _forward(w, "f64", dev)
    ref = og.forward(x, w.kernel, w.ell, w.s, w.sigma2, om_np, A, w.leaf_rows)
    assert int(sol.info.item()) == 0 and ref["info"] == 0
    ex = rel_max(sol.X.cpu().numpy(), ref["X"])
    el = abs(sol.logdet.item() - ref["logdet"]) / abs(ref["logdet"])
    note(f"  X rel {ex:.2e} logdet rel {el:.2e}")
    assert ex <= 1e-10 and el <= 1e-10


def test_c1_fp64_error_against_exact_dense():
    """The method's own error at the plain FP64 workload: the GPU's X~ against
    the exact K^-1 A (dense Cholesky of K_f + sigma2 I on the host). The GPU
    path equals the oracle to 1e-10, so its error against the exact solve is
    the oracle's, stored in tests/golden/exact_dense_reference.txt."""
    from conftest import read_golden
    from oracle import kernels as okr

    gold = {k: float(v) for k, v in read_golden("exact_dense_reference.txt")}
    dev = device()
    w = W.WORKLOADS["C1"]
    x, A, om_np, _, Y, Q, R, sol = _forward(w, "f64", dev)
    xd = x.astype(np.float64)
    k = okr.kernel_matrix(w.kernel, xd, xd, w.ell, w.s) + w.sigma2 * np.eye(w.n)
    lo = np.linalg.cholesky(k)
    xe = np.linalg.solve(lo.T, np.linalg.solve(lo, A.astype(np.float64)))
    err = float(np.linalg.norm(sol.X.cpu().numpy() - xe) / np.linalg.norm(xe))
    ld_ex = 2.0 * float(np.sum(np.log(np.diag(lo))))
    note(f"  X rel error vs exact dense {err:.6e} (method, oracle: {gold['c1_method_x_relerr']:.6e}); "
         f"log|K~| {sol.logdet.item():.10e} vs exact log|K| {ld_ex:.10e}")
    assert abs(err - gold["c1_method_x_relerr"]) <= 1e-8
    assert abs(sol.logdet.item() - gold["c1_method_logdet"]) <= 1e-10 * abs(gold["c1_method_logdet"])


def test_c1_fp64_stagewise_core():
    # the oracle's core and apply fed the GPU's own Q, R (promoted) must agree closely
    dev = device()
    w = W.WORKLOADS["C1"]
    x, A, om_np, _, Y, Q, R, sol = _forward(w, "f64", dev)
    q, r = Q.cpu().numpy(), R.cpu().numpy()
    c = olr.core(q, r, om_np, w.sigma2)
    np.testing.assert_allclose(sol.C.cpu().numpy(), c["C"], rtol=0, atol=1e-9 * np.abs(c["C"]).max())
    np.testing.assert_allclose(sol.L.cpu().numpy(), c["L"], rtol=0, atol=1e-9 * np.abs(c["L"]).max())
    xr = olr.apply(q, c["L"], A, w.sigma2)
    assert rel_max(sol.X.cpu().numpy(), xr) <= 1e-12


@pytest.mark.parametrize("nu", [0.0, 0.02])
def test_gauss_fp64_small_with_shift(nu):
    dev = device()
    w = W.small(W.WORKLOADS["C3"], 2500, d=96, leaf_rows=600, m=3).replace(ell=0.25, sigma2=1e-2)
    x, A, om_np, _, Y, Q, R, sol = _forward(w.replace(prec="f64"), "f64", dev, nu=nu)
    ref = og.forward(x, w.kernel, w.ell, w.s, w.sigma2, om_np, A, w.leaf_rows, nu=nu)
    ex = rel_max(sol.X.cpu().numpy(), ref["X"])
    el = abs(sol.logdet.item() - ref["logdet"]) / abs(ref["logdet"])
    note(f"  X rel {ex:.2e} logdet rel {el:.2e}")
    assert ex <= 1e-10 and el <= 1e-10


def test_gauss_fp64_largest_d():
    """d = 1024, the largest rank the boundary takes: 1024-thread LU and
    Cholesky panels and tree panels with several rows per thread. Reference:
    the oracle's sketch and Woodbury solve around the unique positive-diagonal
    QR of Y (LAPACK's, sign-fixed; the oracle's own column-by-column QR needs
    tens of seconds at this size)."""
    dev = device()
    w = W.small(W.WORKLOADS["C3"], 2048, d=1024, leaf_rows=1024, m=2).replace(ell=0.1, sigma2=1e-1)
    x, A, om_np, _, Y, Q, R, sol = _forward(w.replace(prec="f64"), "f64", dev)
    y = osk.sketch(x, w.kernel, w.ell, w.s, om_np)
    q, r = np.linalg.qr(y)
    sg = np.where(np.diag(r) < 0, -1.0, 1.0)
    ref = olr.solve(q * sg[None, :], r * sg[:, None], om_np, w.sigma2, A)
    ex = rel_max(sol.X.cpu().numpy(), ref["X"])
    el = abs(sol.logdet.item() - ref["logdet"]) / abs(ref["logdet"])
    note(f"  X rel {ex:.2e} logdet rel {el:.2e}")
    assert int(sol.info.item()) == 0
    assert ex <= 1e-10 and el <= 1e-10


def _model_forward(x, w, om_np, A, y_model):
    q, r = qr_fp32(y_model)
    return olr.solve(q, r, om_np, w.sigma2, A)


def test_srht_fp32_path_error_vs_fp64_oracle():
    dev = device()
    w = W.small(W.WORKLOADS["C2"], 16384, d=128, leaf_rows=4096)
    x, A, om_np, _, Y, Q, R, sol = _forward(w, "f32", dev)
    ref = og.forward(x, w.kernel, w.ell, w.s, w.sigma2, om_np, A, w.leaf_rows)
    mod = _model_forward(x, w, om_np, A, Y.double().cpu().numpy())
    ex = rel_max(sol.X.cpu().numpy(), ref["X"])
    el = abs(sol.logdet.item() - ref["logdet"]) / abs(ref["logdet"])
    mx = rel_max(mod["X"], ref["X"])
    ml = abs(mod["logdet"] - ref["logdet"]) / abs(ref["logdet"])
    note(f"  FP32 path: X rel {ex:.2e} logdet rel {el:.2e}; float32 model X {mx:.2e} logdet {ml:.2e}")
    assert ex <= 1e-5 + 4.0 * mx and el <= 1e-8 + 4.0 * ml


def test_bf16_path_error_vs_fp64_oracle():
    dev = device()
    w = W.small(W.WORKLOADS["C3"], 4096, d=128, leaf_rows=1024, m=4)
    x, A, om_np, _, Y, Q, R, sol = _forward(w, "bf16", dev)
    ref = og.forward(x, w.kernel, w.ell, w.s, w.sigma2, om_np, A, w.leaf_rows)
    refb = og.forward(x, w.kernel, w.ell, w.s, w.sigma2, om_np, A, w.leaf_rows, k_round="bf16")
    # precision model: the GPU's sketch (float32-evaluated kernel entries
    # rounded to bf16, float32 sums), LAPACK's float32 QR, float64 core
    mod = _model_forward(x, w, om_np, A, Y.double().cpu().numpy())
    ex = rel_max(sol.X.cpu().numpy(), ref["X"])
    exb = rel_max(sol.X.cpu().numpy(), refb["X"])
    el = abs(sol.logdet.item() - ref["logdet"]) / abs(ref["logdet"])
    elb = abs(sol.logdet.item() - refb["logdet"]) / abs(refb["logdet"])
    mx = rel_max(mod["X"], refb["X"])
    ml = abs(mod["logdet"] - refb["logdet"]) / abs(refb["logdet"])
    note(f"  BF16 path: X rel vs fp64 {ex:.2e}, vs bf16-K oracle {exb:.2e} (float32 model {mx:.2e}); "
         f"logdet rel {el:.2e}, vs bf16-K oracle {elb:.2e} (model {ml:.2e})")
    # the bf16 rounding of K itself (G12 of the design notes: X moves by ~3e-2)
    assert ex <= 5e-2 and el <= 2e-4
    # against the oracle that rounds K to bf16 as the kernel does
    assert exb <= 1e-5 + 4.0 * mx and elb <= 1e-8 + 4.0 * ml


def test_bf16x2_path_error_vs_fp64_oracle():
    """The two-term bf16 sketch: K carried to 16 bits (the oracle's bf16x2
    precision model), float32 leaf QR, float64 tree and core."""
    dev = device()
    w = W.small(W.WORKLOADS["C3"], 4096, d=128, leaf_rows=1024, m=4)
    x, A, om_np, _, Y, Q, R, sol = _forward(w, "bf16x2", dev)
    ref = og.forward(x, w.kernel, w.ell, w.s, w.sigma2, om_np, A, w.leaf_rows)
    refb = og.forward(x, w.kernel, w.ell, w.s, w.sigma2, om_np, A, w.leaf_rows, k_round="bf16x2")
    mod = _model_forward(x, w, om_np, A, Y.double().cpu().numpy())
    ex = rel_max(sol.X.cpu().numpy(), ref["X"])
    exb = rel_max(sol.X.cpu().numpy(), refb["X"])
    el = abs(sol.logdet.item() - ref["logdet"]) / abs(ref["logdet"])
    mx = rel_max(mod["X"], ref["X"])
    ml = abs(mod["logdet"] - ref["logdet"]) / abs(ref["logdet"])
    note(f"  BF16X2 path: X rel vs fp64 {ex:.2e} (vs bf16x2-K oracle {exb:.2e}; float32 model {mx:.2e}), "
         f"logdet rel {el:.2e} (model {ml:.2e})")
    assert ex <= 1e-5 + 4.0 * mx and el <= 1e-8 + 4.0 * ml


def test_not_pd_reports_info_and_leaves_x():
    dev = device()
    a = api()
    w = W.small(W.WORKLOADS["C1"], 512, d=16, leaf_rows=64, m=2)
    x, A, om_np, om, Y, Q, R, sol = _forward(w, "f64", dev)
    c = sol.C.cpu().numpy()
    nu = w.sigma2 + np.linalg.eigvalsh(c).min() + 1.0
    Ad = to_dev(A, torch.float64, dev)
    bad = a.lowrank_solve(Q, R, om, "f64", w.sigma2, Ad, nu=nu)
    torch.cuda.synchronize()
    assert int(bad.info.item()) > 0 and math.isnan(bad.logdet.item())


def test_m_zero_computes_logdet_only():
    dev = device()
    a = api()
    w = W.WORKLOADS["C1"]
    x, A, om_np, om, Y, Q, R, sol = _forward(w, "f64", dev)
    s0 = a.lowrank_solve(Q, R, om, "f64", w.sigma2, None)
    torch.cuda.synchronize()
    assert s0.X is None and abs(s0.logdet.item() - sol.logdet.item()) <= 1e-12 * abs(sol.logdet.item())


def test_c3_full_bf16_stagewise():
    """Full headline workload (n = 262144, d = 512, Matern-3/2, Gaussian Omega,
    bf16 sketch): the oracle's core and Woodbury solve fed the GPU's own Q and R
    (promoted) against the GPU's C, L, log-det and X. The GPU's F = Omega^T Q
    sums float products in float32 for at most 512 rows (gamma_512 u32 of
    |Omega|^T |Q|, see test_omega_t_q_product_against_oracle); C = F^{-1} R^T
    and the Cholesky factor inherit that relative error times cond(F); X is
    formed in float64 from Z = Q^T A summed exactly and rounded once to float32."""
    dev = device()
    w = W.WORKLOADS["C3"]
    x, A, om_np, om, Y, Q, R, sol = _forward(w, "bf16", dev)
    assert int(sol.info.item()) == 0
    q, r = Q.double().cpu().numpy(), R.cpu().numpy()
    c = olr.core(q, r, om_np, w.sigma2)
    assert c["info"] == 0
    kf = float(np.linalg.cond(c["F"]))
    tol_c = 10.0 * kf * 520 * 2.0 ** -24
    eC = float(np.abs(sol.C.cpu().numpy() - c["C"]).max() / np.abs(c["C"]).max())
    eL = float(np.abs(sol.L.cpu().numpy() - c["L"]).max() / np.abs(c["L"]).max())
    ld = olr.logdet(c["L"], w.n, w.sigma2)
    el = abs(sol.logdet.item() - ld) / abs(ld)
    xr = olr.apply(q, c["L"], A, w.sigma2)
    ex = rel_max(sol.X.double().cpu().numpy(), xr)
    note(f"  C3 stage-wise: C {eC:.2e} L {eL:.2e} logdet {el:.2e} X {ex:.2e} (cond F {kf:.1f}, C/L bar {tol_c:.1e})")
    assert eC <= tol_c and eL <= tol_c
    assert el <= tol_c
    assert ex <= 2.0 ** -24 + float(np.linalg.cond(c["S"])) * tol_c


@pytest.mark.parametrize("prec", ["bf16", "f32"])
def test_omega_t_q_product_against_oracle(prec):
    """F = Omega^T Q (the d x d cross product of the Woodbury core), read back
    from the LU factors lr_lowrank_solve returns, against the FP64 product of
    the same Omega values and the same float32 Q. Ragged n (two full row
    chunks of 4096 plus 40 rows) so every row path of the product is taken.
    Bound: float32 partial sums of at most 512 terms (then float64), i.e.
    gamma_512 u32 relative to sum_r |Omega_ri| |Q_rj|."""
    dev = device()
    a = api()
    n, d, m = 8232, 128, 3
    rng = np.random.default_rng(31)
    q = np.linalg.qr(rng.standard_normal((n, d)))[0].astype(np.float32)
    r = np.triu(rng.standard_normal((d, d)), 1) + np.diag(1.0 + np.abs(rng.standard_normal(d)))
    w = W.small(W.WORKLOADS["C3"], n, d=d, m=m)
    om_np, om = omega_pair(w, prec, dev)
    A = rng.standard_normal((n, m)).astype(np.float32)
    note(f"Omega^T Q product n={n} d={d} prec={prec}")
    sol = a.lowrank_solve(to_dev(q, torch.float32, dev), to_dev(r, torch.float64, dev), om, prec, w.sigma2,
                          to_dev(A, torch.float32, dev))
    torch.cuda.synchronize()
    # random Q, R need not give a positive definite core (info > 0 from the
    # Cholesky); the LU factors of F are written before it (info < 0 would be
    # a zero pivot of F)
    assert int(sol.info.item()) >= 0
    flu = sol.Flu.cpu().numpy()
    piv = sol.piv.cpu().numpy()
    f = (np.tril(flu, -1) + np.eye(d)) @ np.triu(flu)
    for k in range(d - 1, -1, -1):  # undo the row exchanges, last first
        p = int(piv[k])
        f[[k, p]] = f[[p, k]]
    om_t = om_np["omega_t"].astype(np.float64)
    q64 = q.astype(np.float64)
    ref = om_t @ q64
    scale = np.abs(om_t) @ np.abs(q64)
    err = float((np.abs(f - ref) / scale).max())
    note(f"  max |F - Omega^T Q| / (|Omega|^T |Q|) = {err:.3e}")
    assert err <= 520 * 2.0 ** -24


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_srht_omega_t_q_transform_against_oracle(prec):
    """F = Omega^T Q for an SRHT Omega (Def. 1), read back from the LU factors
    as above. n = 16384 with d = 100 (not a multiple of the 64 outputs a lane
    group owns): in float32 the product takes the column-wise fast transform
    over eight 2048-row slabs, in float64 the workspace holds no slab and the
    generated-operand product runs instead. Both sum exact products in float64
    (transform depth log2(2048) plus the chunk and slab sums), so the bar is
    64 u64 relative to sum_r |Omega_ri| |Q_rj| = c sum_r |Q_rj|."""
    dev = device()
    a = api()
    n, d, m = 16384, 100, 3
    rng = np.random.default_rng(37)
    q = np.linalg.qr(rng.standard_normal((n, d)))[0]
    q = q.astype(np.float32).astype(np.float64)
    r = np.triu(rng.standard_normal((d, d)), 1) + np.diag(1.0 + np.abs(rng.standard_normal(d)))
    w = W.small(W.WORKLOADS["C2"], n, d=d, m=m)
    om_np, om = omega_pair(w, prec, dev)
    dt = torch.float64 if prec == "f64" else torch.float32
    A = rng.standard_normal((n, m))
    note(f"SRHT Omega^T Q product n={n} d={d} prec={prec}")
    sol = a.lowrank_solve(to_dev(q, dt, dev), to_dev(r, torch.float64, dev), om, prec, w.sigma2, to_dev(A, dt, dev))
    torch.cuda.synchronize()
    assert int(sol.info.item()) >= 0
    flu = sol.Flu.cpu().numpy()
    piv = sol.piv.cpu().numpy()
    lo, up = np.tril(flu, -1) + np.eye(d), np.triu(flu)
    f, lu_abs = lo @ up, np.abs(lo) @ np.abs(up)
    for k in range(d - 1, -1, -1):
        p = int(piv[k])
        f[[k, p]] = f[[p, k]]
        lu_abs[[k, p]] = lu_abs[[p, k]]
    ref = osk.omega_t_apply(om_np, q)
    scale = np.abs(q).sum(axis=0)[None, :] / np.sqrt(n)
    # product bar plus the float64 LU's backward error and the reconstruction
    # product (gamma_d |L||U| each)
    u = 2.0 ** -53
    bar = 64 * u * scale + 2 * (d + 2) * u * lu_abs
    err = float((np.abs(f - ref) / bar).max())
    note(f"  max |F - Omega^T Q| / bar = {err:.3e}; max error relative to |Omega|^T |Q|: "
         f"{float((np.abs(f - ref) / scale).max()):.3e}")
    assert err <= 1.0


def test_c2_full_fp32_against_fp64_path():
    """The FP32-vs-FP64 workload at full size (n = 65536, D = 3, SE, SRHT
    d = 256, A 65536 x 8). The FP64 path is pinned to the oracle: sketch rows
    sampled against the oracle's (SRHT bar), and the oracle's core and apply
    fed the GPU's FP64 Q and R (1e-10). The FP32 path is compared stage-wise
    the same way (the C/L bar of test_c3_full_bf16_stagewise) and end to end
    with the FP64 path, against 4x the distance of the oracle's float32
    precision model (the GPU's float32 sketch, LAPACK's float32 QR, the float64
    core and apply) from that path."""
    dev = device()
    w = W.WORKLOADS["C2"]
    x, A, om_np, _, Y64, Q64, R64, sol64 = _forward(w, "f64", dev)
    assert int(sol64.info.item()) == 0
    rows = np.concatenate([[0, w.n - 1], np.random.default_rng(5).choice(w.n, 10, replace=False)])
    y_ref = osk.sketch_rows(x, rows, w.kernel, w.ell, w.s, om_np)
    from oracle import kernels as okr
    kabs = np.abs(okr.kernel_matrix(w.kernel, x[rows].astype(np.float64), x.astype(np.float64), w.ell, w.s))
    sc = kabs.sum(axis=1, keepdims=True) / math.sqrt(w.n)
    ey = (np.abs(Y64.cpu().numpy()[rows] - y_ref) / sc).max()
    q64, r64 = Q64.cpu().numpy(), R64.cpu().numpy()
    ref64 = olr.solve(q64, r64, om_np, w.sigma2, A.astype(np.float64))
    ex64 = rel_max(sol64.X.cpu().numpy(), ref64["X"])
    el64 = abs(sol64.logdet.item() - ref64["logdet"]) / abs(ref64["logdet"])
    note(f"  FP64 path: sampled Y {ey:.2e} of the SRHT scale; stage-wise X {ex64:.2e} logdet {el64:.2e}")
    assert ey <= 16 * math.log2(w.n) * 2.0 ** -53
    assert ex64 <= 1e-10 and el64 <= 1e-10
    x32, A32, _, _, Y32, Q32, R32, sol32 = _forward(w, "f32", dev)
    assert int(sol32.info.item()) == 0
    q, r = Q32.double().cpu().numpy(), R32.cpu().numpy()
    c = olr.core(q, r, om_np, w.sigma2)
    assert c["info"] == 0
    kf = float(np.linalg.cond(c["F"]))
    tol_c = 10.0 * kf * 520 * 2.0 ** -24
    eC = float(np.abs(sol32.C.cpu().numpy() - c["C"]).max() / np.abs(c["C"]).max())
    ld = olr.logdet(c["L"], w.n, w.sigma2)
    el = abs(sol32.logdet.item() - ld) / abs(ld)
    xr = olr.apply(q, c["L"], A.astype(np.float64), w.sigma2)
    ex = rel_max(sol32.X.double().cpu().numpy(), xr)
    note(f"  FP32 stage-wise: C {eC:.2e} logdet {el:.2e} X {ex:.2e} (cond F {kf:.1f}, bar {tol_c:.1e})")
    assert eC <= tol_c and el <= tol_c
    assert ex <= 2.0 ** -24 + float(np.linalg.cond(c["S"])) * tol_c
    mod = _model_forward(x, w, om_np, A, Y32.double().cpu().numpy())
    x64 = sol64.X.cpu().numpy()
    d_x = rel_max(sol32.X.double().cpu().numpy(), x64)
    d_l = abs(sol32.logdet.item() - sol64.logdet.item()) / abs(sol64.logdet.item())
    m_x = rel_max(mod["X"], x64)
    m_l = abs(mod["logdet"] - sol64.logdet.item()) / abs(sol64.logdet.item())
    note(f"  FP32 vs FP64 path: X {d_x:.2e} logdet {d_l:.2e}; float32 model X {m_x:.2e} logdet {m_l:.2e}")
    assert d_x <= 1e-5 + 4.0 * m_x and d_l <= 1e-8 + 4.0 * m_l
