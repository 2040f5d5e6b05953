"""GPU parity of lr_backward (hyperparameter adjoint) and the autograd wrappers.

Two kinds of check:

* Stage-wise (isolates lr_backward). The oracle's gradient formulas are fed
  the GPU's own Q (promoted to float64), R, its core factors (LU of F, C, L)
  and its derivative sketch Y'. Both sides then evaluate the same float64
  formulas on the same numbers, so they must agree to float64 rounding
  amplified by the conditioning of the d x d core: 1e-8 of |g| per component
  (every n-length product in lr_backward sums exact products in float64),
  plus cond(S) u64 times the magnitude of the contractions each component
  adds up (_loglik_term_scales; matters at the full log-likelihood workload,
  cond(S) ~ 2e6).
  With a shift the GPU simplifies the projector terms with Q^T Q = I while
  the oracle evaluates them on the float Q as given, so those terms may
  differ by d max|Q^T Q - I| of |g| more (~5e-6 for a float32 Q).
* End to end against the oracle run from scratch. FP64 path: 1e-9 of |g| per
  component. FP32 path: the float32 sketch's error (a few roundings of Y)
  and the backward error of the float32 QR (about u32 ||Y e_j|| per column j,
  against trailing singular values of Y that are only ~1e-5 ||Y|| for the
  squared-exponential kernel) perturb the directions the Nystrom form weights
  most, and the float64 method itself reacts strongly, and differently for
  each perturbation of the same size: LAPACK's own float32 QR moves d/dlog s
  by ~10% at n = 4096, d = 64. The bar samples that reaction. A backward
  stable QR returns the exact QR of Y + E with ||E e_j|| <= beta ||Y e_j||;
  beta is measured on the GPU's Q and R, and the oracle (core and gradient,
  after LAPACK's float64 QR for speed) is run on the GPU's sketch plus 8
  random column-wise perturbations of relative size beta. Per component,
      |g - g_ref| <= 1e-4 |g_ref| + 3 max_k |g(Y_gpu + E_k) - g_ref|.
  For the Matern kernel (well conditioned) the samples move g by < 1e-5 and
  the 1e-4 term binds. A shift nu (Y = (K_f + nu I) Omega, nu ~ sigma2 / 10)
  lifts the trailing directions above float32 resolution and brings the SE
  gradient to a few 1e-4.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import grad as og, lowrank as olr, qr as oqr, sketch as osk

from conftest import read_golden
from gpu_common import api, device, hyper, note, omega_pair, qr_fp64, to_dev, torch

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def _gpu_run(w, prec, dev, A, fused, mode=0, abar=None, nu=0.0):
    """Forward + backward through the C ABI; returns everything the checks need."""
    a = api()
    x = W.points(w)
    om_np, om = omega_pair(w, prec, dev)
    dt = torch.float64 if prec == "f64" else torch.float32
    X = to_dev(x, torch.float32, dev)
    Ad = to_dev(A, dt, dev)
    h = hyper(w)
    fw = a.forward(X, h, om, prec, w.sigma2, Ad, w.leaf_rows, nu=nu, want_yprime=fused)
    yp = fw.Yprime
    if yp is None:
        _, yp = a.sketch(X, h, om, prec, want_y=False, want_yprime=True)
    V = None if abar is None else to_dev(abar, dt, dev)
    dth, dA = a.backward(X, h, om, prec, fw.sol, fw.Q, w.sigma2, mode, Ad, V=V, Yprime=fw.Yprime,
                         want_dA=abar is not None, R=fw.R, nu=nu)
    torch.cuda.synchronize()
    assert int(fw.sol.info.item()) == 0
    core = {"lu": (fw.sol.Flu.cpu().numpy(), fw.sol.piv.cpu().numpy().astype(np.int32)),
            "C": fw.sol.C.cpu().numpy(), "L": fw.sol.L.cpu().numpy()}
    return {"x": x, "om": om_np, "Y": fw.Y.double().cpu().numpy(), "Q": fw.Q.double().cpu().numpy(),
            "R": fw.R.cpu().numpy(),
            "Yp": yp.double().cpu().numpy(), "core": core, "g": dth.cpu().numpy(),
            "dA": None if dA is None else dA.double().cpu().numpy(), "sol": fw.sol,
            "X": fw.sol.X.double().cpu().numpy(), "logdet": fw.sol.logdet.item()}


def _oracle_loglik_grad(x, w, om, yv, y, yp, nu=0.0, lapack=False):
    q, r = qr_fp64(y) if lapack else oqr.tsqr(y, w.leaf_rows)
    core = olr.solve(q, r, om, w.sigma2, yv.reshape(-1, 1), nu)
    assert core["info"] == 0
    ll = olr.loglik(yv, core["X"][:, 0], core["logdet"])
    return og.grad_loglik(x, w.kernel, w.ell, w.s, w.sigma2, om, q, core, yv, yprime=yp, nu=nu, r=r), ll


def _stage_bar(q, nu):
    d = q.shape[1]
    orth = float(np.abs(q.T @ q - np.eye(d)).max()) if nu != 0.0 else 0.0
    return 1e-8 + d * orth


def _loglik_term_scales(r, yv, sigma2):
    """Per component, the magnitudes of the d x d contractions lr_backward adds
    up for the log-likelihood (u.h, <S^-1 Phi, P>, u.E u, <Phi^T S^-1 Phi, E>;
    a.C a, <S^-1, C>; alpha^T alpha, (n - d)/sigma2, tr S^-1), and cond(S).
    S^-1 and Phi = F^-1 enter every one of them, and two implementations of
    the solves differ by about cond(S) u64 relative, so the stage-wise gap of
    component k can reach cond(S) u64 times its scale."""
    q, core, yp = r["Q"], r["core"], r["Yp"]
    n, d = q.shape
    L = core["L"]
    s_inv = olr.s_solve(L, np.eye(d))
    flu, piv = core["lu"]
    import scipy.linalg as sla
    phi = sla.lu_solve((flu, piv), np.eye(d))
    y = yv.astype(np.float64)
    a = olr.s_solve(L, q.T @ y)
    alpha = olr.apply(q, L, y.reshape(-1, 1), sigma2)[:, 0]
    u = phi.T @ a
    h = yp.T @ alpha
    p_ = q.T @ yp
    e_ = osk.omega_t_apply(r["om"], yp)
    t_ = s_inv @ phi
    g2 = phi.T @ t_
    m_ell = abs(u @ h) + abs(np.sum(t_ * p_)) + 0.5 * (abs(u @ e_ @ u) + abs(np.sum(g2 * e_)))
    m_s = abs(a @ core["C"] @ a) + abs(np.sum(s_inv * core["C"]))
    m_sig = 0.5 * sigma2 * (alpha @ alpha + (n - d) / sigma2 + abs(np.trace(s_inv)))
    return np.array([m_ell, m_s, m_sig]), float(np.linalg.cond(L @ L.T))


def _loglik_stage_bar(r, yv, sigma2, g_st, nu):
    m, cond_s = _loglik_term_scales(r, yv, sigma2)
    return _stage_bar(r["Q"], nu) * np.abs(g_st) + 8.0 * cond_s * 2.0 ** -53 * m


def _perturbed(y, beta, k, seed=7):
    """y plus a random perturbation of relative size beta in every column."""
    rng = np.random.default_rng(seed + k)
    e = rng.standard_normal(y.shape)
    e *= beta * np.linalg.norm(y, axis=0) / np.linalg.norm(e, axis=0)
    return y + e


def _fp32_bar(g_ref, g_samples):
    dev = np.max(np.abs(np.asarray(g_samples) - g_ref[None, :]), axis=0)
    return 1e-4 * np.abs(g_ref) + 3.0 * dev


def _qr_backward_errors(y, q, r):
    """max over columns of ||(Q R - Y) e_j|| / ||Y e_j||, and ||Q^T Q - I||_max."""
    res = np.linalg.norm(q @ r - y, axis=0) / np.maximum(np.linalg.norm(y, axis=0), 1e-300)
    return float(res.max()), float(np.abs(q.T @ q - np.eye(q.shape[1])).max())


@pytest.mark.parametrize("prec,kind,fused,nu_frac", [("f64", "se", False, 0.0), ("f32", "se", True, 0.0),
                                                     ("f64", "matern32", False, 0.0), ("f32", "matern32", False, 0.0),
                                                     ("f64", "se", False, 0.1), ("f32", "se", True, 0.1),
                                                     ("f64", "matern32", True, 0.5)])
def test_loglik_gradient(prec, kind, fused, nu_frac):
    dev = device()
    w = W.small(W.WORKLOADS["C4"], 4096, d=64, leaf_rows=1024).replace(kernel=kind)
    nu = nu_frac * w.sigma2
    x = W.points(w)
    yv = W.gp_targets(w, x)
    note(f"loglik grad {kind} prec={prec} fused={fused} nu={nu} n={w.n} d={w.d}")
    r = _gpu_run(w, prec, dev, yv.reshape(-1, 1), fused, nu=nu)
    # stage-wise: the oracle's formulas on the GPU's Q, R, factors and Y'
    g_st = og.grad_loglik(x, kind, w.ell, w.s, w.sigma2, r["om"], r["Q"], r["core"], yv, yprime=r["Yp"], nu=nu,
                          r=r["R"])
    e_st = _rel(r["g"], g_st)
    # end to end: the oracle from scratch
    y_ref = osk.sketch(x, kind, w.ell, w.s, r["om"], nu=nu)
    yp_ref = osk.sketch(x, kind, w.ell, w.s, r["om"], deriv=True)
    g_ref, ll_ref = _oracle_loglik_grad(x, w, r["om"], yv, y_ref, yp_ref, nu=nu)
    e_e2e = _rel(r["g"], g_ref)
    sbar = _loglik_stage_bar(r, yv, w.sigma2, g_st, nu)
    note(f"  grad {r['g']} stage-wise rel {e_st} (bar {sbar / np.abs(g_st)}) end-to-end rel {e_e2e} ref {g_ref}")
    assert np.all(np.abs(r["g"] - g_st) <= sbar)
    if prec == "f64":
        assert np.all(e_e2e <= 1e-9)
    else:
        beta, orth = _qr_backward_errors(r["Y"], r["Q"], r["R"])
        g_s = [_oracle_loglik_grad(x, w, r["om"], yv, _perturbed(r["Y"], beta, k), r["Yp"], nu=nu, lapack=True)[0]
               for k in range(8)]
        bar = _fp32_bar(g_ref, g_s)
        note(f"  QR backward error {beta:.2e}; perturbed samples move g by up to "
             f"{np.max(np.abs(np.array(g_s) - g_ref), axis=0) / np.abs(g_ref)}; bar/|g| {bar / np.abs(g_ref)}")
        assert np.all(np.abs(r["g"] - g_ref) <= bar)


def test_loglik_autograd_matches_abi():
    """LowRankLogLik.apply / backward give the same numbers as the ABI calls."""
    dev = device()
    from paper_1312_1869_amd import autograd as ag

    w = W.small(W.WORKLOADS["C4"], 2048, d=32, leaf_rows=512)
    x = W.points(w)
    yv = W.gp_targets(w, x)
    om_np, om = omega_pair(w, "f64", dev)
    theta = torch.tensor([math.log(w.ell), math.log(w.s), math.log(w.sigma2)], dtype=torch.float64,
                         requires_grad=True)
    cfg = ag.Config(w.kernel, "f64", w.leaf_rows)
    ll = ag.LowRankLogLik.apply(theta, to_dev(yv, torch.float64, dev), to_dev(x, torch.float32, dev), om, cfg)
    (g,) = torch.autograd.grad(ll, theta)
    r = _gpu_run(w, "f64", dev, yv.reshape(-1, 1).astype(np.float64), False)
    note(f"  autograd {g.numpy()} abi {r['g']}")
    np.testing.assert_allclose(g.numpy(), r["g"], rtol=1e-12)


@pytest.mark.parametrize("prec,nu_frac", [("f64", 0.0), ("f32", 0.0), ("f64", 0.3), ("f32", 0.3)])
def test_solve_vjp(prec, nu_frac):
    dev = device()
    w = W.small(W.WORKLOADS["C4"], 2048, d=48, leaf_rows=512, m=3)
    nu = nu_frac * w.sigma2
    x = W.points(w)
    A = W.rhs(w)
    abar = np.random.default_rng(3).standard_normal(A.shape).astype(np.float32)
    note(f"solve vjp prec={prec} nu={nu}")
    r = _gpu_run(w, prec, dev, A, False, mode=1, abar=abar, nu=nu)
    g_st, b_st = og.grad_solve(x, w.kernel, w.ell, w.s, w.sigma2, r["om"], r["Q"], r["core"], A, abar,
                               yprime=r["Yp"], nu=nu, r=r["R"])
    e_st = _rel(r["g"], g_st)
    e_b = float(np.abs(r["dA"] - b_st).max() / np.abs(b_st).max())
    f = og.forward(x, w.kernel, w.ell, w.s, w.sigma2, r["om"], A, w.leaf_rows, nu=nu)
    g_ref, b_ref = og.grad_solve(x, w.kernel, w.ell, w.s, w.sigma2, r["om"], f["Q"], f, A, abar, nu=nu, r=f["R"])
    e_e2e = _rel(r["g"], g_ref)
    e_a = float(np.abs(r["dA"] - b_ref).max() / np.abs(b_ref).max())
    note(f"  dtheta {r['g']} stage-wise rel {e_st} end-to-end rel {e_e2e}; dA vs stage-wise {e_b:.2e}, "
         f"vs oracle {e_a:.2e}")
    assert np.all(e_st <= _stage_bar(r["Q"], nu))
    # dA = B rounded once to the working precision
    assert e_b <= (1e-12 if prec == "f64" else 2.0 ** -23)
    if prec == "f64":
        assert np.all(e_e2e <= 1e-9) and e_a <= 1e-10
    else:
        beta, orth = _qr_backward_errors(r["Y"], r["Q"], r["R"])
        g_s, b_s = [], []
        for k in range(8):
            qk, rk = qr_fp64(_perturbed(r["Y"], beta, k))
            fk = olr.solve(qk, rk, r["om"], w.sigma2, A, nu)
            gk, bk = og.grad_solve(x, w.kernel, w.ell, w.s, w.sigma2, r["om"], qk, fk, A, abar, yprime=r["Yp"],
                                   nu=nu, r=rk)
            g_s.append(gk)
            b_s.append(bk)
        bar = _fp32_bar(g_ref, g_s)
        e_am = max(float(np.abs(bk - b_ref).max() / np.abs(b_ref).max()) for bk in b_s)
        note(f"  QR backward error {beta:.2e}; perturbed samples move g by up to "
             f"{np.max(np.abs(np.array(g_s) - g_ref), axis=0) / np.abs(g_ref)}, dA by {e_am:.2e}; "
             f"bar/|g| {bar / np.abs(g_ref)}")
        assert np.all(np.abs(r["g"] - g_ref) <= bar)
        assert e_a <= 1e-5 + 3.0 * e_am


def _golden_c4():
    return {k: float(v) for k, v in read_golden("c4_oracle_reference.txt")}


def _golden_exact():
    return {k: float(v) for k, v in read_golden("exact_dense_reference.txt")}


def test_c4_full_fp32_without_shift_breaks_down_like_the_model():
    """The full log-likelihood workload at FP32 with nu = 0: the trailing
    singular values of the sketch (~1e-15 of the largest for this kernel and
    d = 256) sit far below float32 resolution, so the float32 QR's rounding
    leaves C indefinite and the Cholesky of S = C + sigma2 I fails. The
    oracle's float32 precision model (float32 sketch, LAPACK float32 QR)
    breaks down the same way (tests/golden/c4_oracle_reference.txt); both
    report the failing pivot instead of returning a number."""
    dev = device()
    a = api()
    w = W.WORKLOADS["C4"]
    x = W.points(w)
    yv = W.gp_targets(w, x)
    gold = _golden_c4()
    om_np, om = omega_pair(w, "f32", dev)
    note("C4 full fp32 nu=0")
    fw = a.forward(to_dev(x, torch.float32, dev), hyper(w), om, "f32", w.sigma2,
                   to_dev(yv.reshape(-1, 1), torch.float32, dev), w.leaf_rows)
    torch.cuda.synchronize()
    info = int(fw.sol.info.item())
    note(f"  GPU info {info}, oracle float32 model info {int(gold['info_fp32model'])}, oracle info {int(gold['info'])}")
    assert int(gold["info"]) == 0 and int(gold["info_fp32model"]) > 0
    assert info > 0 and math.isnan(fw.sol.logdet.item())


def test_c4_full_fp32_shifted_loglik_and_gradient():
    """The full log-likelihood workload at its own precision (FP32, n = 32768,
    d = 256) with the stabilising shift nu = sigma2 / 10: stage-wise against the
    oracle's formulas fed the GPU's Q, R, factors and Y'; end to end against
    the stored FP64 oracle values at the same shift
    (tests/golden/c4_oracle_reference.txt). The targets are the seeded
    random-Fourier-feature GP draw of workloads.gp_targets."""
    dev = device()
    w = W.WORKLOADS["C4"]
    x = W.points(w)
    yv = W.gp_targets(w, x)
    gold = _golden_c4()
    nu = gold["nu"]
    note(f"C4 full fp32 n={w.n} d={w.d} nu={nu} (targets: random-Fourier-feature GP draw)")
    r = _gpu_run(w, "f32", dev, yv.reshape(-1, 1), True, nu=nu)
    ll = -0.5 * float(yv.astype(np.float64) @ r["X"][:, 0]) - 0.5 * r["logdet"]
    g_st = og.grad_loglik(x, w.kernel, w.ell, w.s, w.sigma2, r["om"], r["Q"], r["core"], yv, yprime=r["Yp"], nu=nu,
                          r=r["R"])
    e_st = _rel(r["g"], g_st)
    keys = ["grad_logell", "grad_logs", "grad_logsigma2"]
    g_ref = np.array([gold[k + "_nu"] for k in keys])
    beta, orth = _qr_backward_errors(r["Y"], r["Q"], r["R"])
    samples = [_oracle_loglik_grad(x, w, r["om"], yv, _perturbed(r["Y"], beta, k), r["Yp"], nu=nu, lapack=True)
               for k in range(8)]
    g_s = [g for g, _ in samples]
    e_ll = abs(ll - gold["loglik_nu"]) / abs(gold["loglik_nu"])
    m_ll = max(abs(lk - gold["loglik_nu"]) for _, lk in samples) / abs(gold["loglik_nu"])
    e_e2e = _rel(r["g"], g_ref)
    bar = _fp32_bar(g_ref, g_s)
    note(f"  grad {r['g']} stage-wise rel {e_st}; oracle {g_ref}; end-to-end rel {e_e2e}")
    note(f"  QR backward error {beta:.2e}; perturbed samples move g by up to "
         f"{np.max(np.abs(np.array(g_s) - g_ref), axis=0) / np.abs(g_ref)}; bar/|g| {bar / np.abs(g_ref)}")
    note(f"  loglik {ll:.10e} oracle {gold['loglik_nu']:.10e} rel {e_ll:.2e} (samples up to {m_ll:.2e})")
    sbar = _loglik_stage_bar(r, yv, w.sigma2, g_st, nu)
    note(f"  stage-wise bar/|g| {sbar / np.abs(g_st)}")
    ex = _golden_exact()
    g_ex = np.array([ex["c4_" + k + "_exact"] for k in keys])
    note(f"  against the exact dense log-likelihood (the shift is a change of method): ll error "
         f"{ll - ex['c4_loglik_exact']:.3e} (FP64 oracle at the same shift "
         f"{gold['loglik_nu'] - ex['c4_loglik_exact']:.3e}); grad error {r['g'] - g_ex} (oracle {g_ref - g_ex})")
    assert np.all(np.abs(r["g"] - g_st) <= sbar)
    assert np.all(np.abs(r["g"] - g_ref) <= bar)
    assert e_ll <= 1e-6 + 3.0 * m_ll


def test_c4_full_fp64_gradient():
    """The full log-likelihood workload in FP64: stage-wise (the oracle's
    formulas on the GPU's Q, R, factors and Y'), against central finite
    differences of the GPU's own log-likelihood, and against the stored oracle
    with the sampled-perturbation bar of the module docstring (the trailing
    singular values of this sketch are ~1e-15 of the largest, so even float64
    QRs of the same sketch move d/dlog ell by ~1e-6)."""
    dev = device()
    a = api()
    w = W.WORKLOADS["C4"]
    x = W.points(w)
    yv = W.gp_targets(w, x)
    gold = _golden_c4()
    note("C4 full fp64 gradient")
    r = _gpu_run(w, "f64", dev, yv.reshape(-1, 1).astype(np.float64), False)
    g = r["g"]
    g_st = og.grad_loglik(x, w.kernel, w.ell, w.s, w.sigma2, r["om"], r["Q"], r["core"], yv, yprime=r["Yp"])
    e_st = _rel(g, g_st)
    keys = ["grad_logell", "grad_logs", "grad_logsigma2"]
    g_ref = np.array([gold[k] for k in keys])
    g_lap = np.array([gold[k + "_f64lapack"] for k in keys])
    # with trailing singular values at ~1e-15 the factors satisfy the identities
    # the formulas rely on (Q^T Q = I, C = sym(F^-1 R^T)) only to round-off
    # amplified by that conditioning, so two evaluations of the formulas on the
    # same factors may differ by as much as two float64 QRs of the same sketch
    # move the oracle's gradient (the stored LAPACK-QR run)
    sbar = np.maximum(_loglik_stage_bar(r, yv, w.sigma2, g_st, 0.0), 4.0 * np.abs(g_lap - g_ref))
    om_np, om = omega_pair(w, "f64", dev)
    X = to_dev(x, torch.float32, dev)
    y = to_dev(yv, torch.float64, dev).reshape(-1, 1)
    th0 = np.log([w.ell, w.s, w.sigma2])

    def ll_at(th):
        h = a.Hyper(w.kernel, math.exp(th[0]), math.exp(th[1]))
        fw = a.forward(X, h, om, "f64", math.exp(th[2]), y, w.leaf_rows)
        return a.loglik(y, fw.sol.X, fw.sol.logdet, fw.sol.info, "f64").item()

    ll0 = ll_at(th0)
    # central differences with one Richardson step: truncation O(h^4) is ~1e-8
    # here; rounding of the float64 log-likelihood (|ll| ~ 1e5, ~1e-14 relative)
    # divided by h gives ~1e-6 absolute.
    fd = np.zeros(3)
    h = 2e-3
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        d1 = (ll_at(th0 + h * e) - ll_at(th0 - h * e)) / (2 * h)
        d2 = (ll_at(th0 + 0.5 * h * e) - ll_at(th0 - 0.5 * h * e)) / h
        fd[k] = (4 * d2 - d1) / 3
    beta, orth = _qr_backward_errors(r["Y"], r["Q"], r["R"])
    g_s = [_oracle_loglik_grad(x, w, r["om"], yv, _perturbed(r["Y"], beta, k), r["Yp"], lapack=True)[0]
           for k in range(8)]
    bar = 1e-10 * np.abs(g_ref) + 3.0 * np.max(np.abs(np.array(g_s) - g_ref), axis=0)
    note(f"  ll {ll0:.10e} (oracle {gold['loglik']:.10e}) grad {g} stage-wise rel {e_st} "
         f"(bar {sbar / np.abs(g_st)})")
    note(f"  fd {fd} oracle {g_ref} rel vs oracle {_rel(g, g_ref)} QR backward error {beta:.2e} "
         f"bar/|g| {bar / np.abs(g_ref)}")
    ex = _golden_exact()
    g_ex = np.array([ex["c4_" + k + "_exact"] for k in keys])
    note(f"  against the exact dense log-likelihood: ll error {ll0 - ex['c4_loglik_exact']:.3e} "
         f"(oracle {gold['loglik'] - ex['c4_loglik_exact']:.3e}); grad error {g - g_ex} (oracle {g_ref - g_ex})")
    assert np.all(np.abs(g - g_st) <= sbar)
    assert np.all(np.abs(g - fd) <= 1e-7 * np.abs(g) + 2e-9 * abs(ll0) / h)
    assert abs(ll0 - gold["loglik"]) <= 1e-10 * abs(gold["loglik"])
    assert np.all(np.abs(g - g_ref) <= bar)
    # the method itself (rank 256, no shift) is within 1e-11 of the exact
    # log-likelihood and 3e-6 of its gradient here; the GPU adds at most its
    # parity bars to that
    assert abs(ll0 - ex["c4_loglik_exact"]) <= 1e-11 * abs(ex["c4_loglik_exact"]) + 1e-10 * abs(gold["loglik"])
    assert np.all(np.abs(g - g_ex) <= 3e-6 * np.abs(g_ex) + bar)


def test_c5_full_fused_forward_backward_stagewise():
    """The largest workload at full size (n = 2^20, d = 1024, SE, SRHT, FP32,
    A 2^20 x 16): the fused forward (Y and Y' from one pass) and the backward of
    <A, K~^{-1} A>, stage-wise against the oracle's gradient formulas fed the
    GPU's Q (promoted), core factors and Y' (the bar of the other stage-wise
    checks), and X against the oracle's apply on the same factors. The
    sketch's own parity at this size is test_gpu_sketch's sampled-row check."""
    dev = device()
    w = W.WORKLOADS["C5"]
    A = W.rhs(w)
    note(f"C5 full fused forward + backward n={w.n} d={w.d} m={w.m}")
    r = _gpu_run(w, "f32", dev, A, True, mode=1, abar=A)
    q = r["Q"]
    g_st, _ = og.grad_solve(r["x"], w.kernel, w.ell, w.s, w.sigma2, r["om"], q, r["core"], A, A, yprime=r["Yp"])
    e_st = _rel(r["g"], g_st)
    x_st = olr.apply(q, r["core"]["L"], A.astype(np.float64), w.sigma2)
    ex = float(np.abs(r["X"] - x_st).max() / np.abs(x_st).max())
    note(f"  grad {r['g']} stage-wise {g_st} rel {e_st}; X stage-wise {ex:.2e}")
    assert np.all(e_st <= _stage_bar(q, 0.0))
    assert ex <= 1e-5
