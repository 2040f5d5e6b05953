"""GPU parity of lr_backward (hyperparameter adjoint) and the autograd wrappers.

Expected gradients come from the oracle (Q-basis formulas, pinned there
against finite differences and the dense product rule). Errors are measured
against the magnitude of the terms each component adds up (d/dlog s, for
example, is alpha^T y - sigma2 alpha^T alpha - n + sigma2 tr K~^{-1}, an O(1)
difference of O(n) terms): FP64 path 1e-9 of that scale; FP32 path
4e-3 + 8 u32 cond(S) (float32 Q and sketch satisfy the identities the adjoint
relies on only to O(u32), amplified by the conditioning of S). At the full C4 size, where the FP64 oracle would
need hours, the FP64 GPU gradient is checked against central finite
differences of the GPU's own log-likelihood (a property that holds at any size).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import grad as og

from gpu_common import U32, api, device, hyper, note, omega_pair, to_dev, torch

pytestmark = pytest.mark.gpu


def _setup(w, prec, dev):
    x = W.points(w)
    yv = W.gp_targets(w, x)
    om_np, om = omega_pair(w, prec, dev)
    return x, yv, om_np, om


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


@pytest.mark.parametrize("prec,kind,fused", [("f64", "se", False), ("f32", "se", True), ("f64", "matern32", False),
                                             ("f32", "matern32", False)])
def test_loglik_gradient_matches_oracle(prec, kind, fused):
    dev = device()
    from paper_1312_1869_amd import autograd as ag

    w = W.small(W.WORKLOADS["C4"], 4096, d=64, leaf_rows=1024).replace(kernel=kind)
    x, yv, om_np, om = _setup(w, prec, dev)
    dt = torch.float64 if prec == "f64" else torch.float32
    theta = torch.tensor([math.log(w.ell), math.log(w.s), math.log(w.sigma2)], dtype=torch.float64,
                         requires_grad=True)
    cfg = ag.Config(kind, prec, w.leaf_rows, fused=fused)
    note(f"loglik grad {kind} prec={prec} fused={fused}")
    ll = ag.LowRankLogLik.apply(theta, to_dev(yv, dt, dev), to_dev(x, torch.float32, dev), om, cfg)
    (g,) = torch.autograd.grad(ll, theta)
    f = og.forward(x, kind, w.ell, w.s, w.sigma2, om_np, yv.reshape(-1, 1), w.leaf_rows)
    ref, scale = og.grad_loglik(x, kind, w.ell, w.s, w.sigma2, om_np, f["Q"], f, yv, f["X"][:, 0], parts=True)
    ya = float(yv.astype(np.float64) @ f["X"][:, 0])
    ll_ref = -0.5 * ya - 0.5 * f["logdet"]
    e_ll = abs(ll.item() - ll_ref) / (0.5 * abs(ya) + 0.5 * abs(f["logdet"]))
    e_g = float(np.max(np.abs(g.numpy() - ref) / scale))
    cond_s = float(np.linalg.cond(f["S"]))
    note(f"  loglik err/scale {e_ll:.2e}  grad err/scale {e_g:.2e}  cond(S) {cond_s:.2e}  grad {g.numpy()} "
         f"ref {ref} scale {scale}")
    assert e_ll <= (1e-10 if prec == "f64" else 1e-4)
    # float32 Q satisfies Q^T Q = I and F R = Omega^T Y only to O(u32); S^{-1}
    # enters the adjoint, so its conditioning amplifies that
    assert e_g <= (1e-9 if prec == "f64" else 8 * U32 * cond_s + 4e-3)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_solve_vjp_matches_oracle(prec):
    dev = device()
    from paper_1312_1869_amd import autograd as ag

    w = W.small(W.WORKLOADS["C4"], 2048, d=48, leaf_rows=512, m=3)
    x, yv, om_np, om = _setup(w, prec, dev)
    A = W.rhs(w)
    abar = np.random.default_rng(3).standard_normal(A.shape).astype(np.float32)
    dt = torch.float64 if prec == "f64" else torch.float32
    theta = torch.tensor([math.log(w.ell), math.log(w.s), math.log(w.sigma2)], dtype=torch.float64,
                         requires_grad=True)
    Ad = to_dev(A, dt, dev).requires_grad_(True)
    cfg = ag.Config(w.kernel, prec, w.leaf_rows)
    note(f"solve vjp prec={prec}")
    X = ag.LowRankSolve.apply(theta, Ad, to_dev(x, torch.float32, dev), om, cfg)
    gt, gA = torch.autograd.grad(X, (theta, Ad), grad_outputs=to_dev(abar, dt, dev))
    f = og.forward(x, w.kernel, w.ell, w.s, w.sigma2, om_np, A, w.leaf_rows)
    ref, b, scale = og.grad_solve(x, w.kernel, w.ell, w.s, w.sigma2, om_np, f["Q"], f, f["X"], abar, parts=True)
    e_g = float(np.max(np.abs(gt.numpy() - ref) / scale))
    e_a = float(np.abs(gA.double().cpu().numpy() - b).max() / np.abs(b).max())
    cond_s = float(np.linalg.cond(f["S"]))
    note(f"  dtheta err/scale {e_g:.2e}  dA rel {e_a:.2e}  cond(S) {cond_s:.2e}  grad {gt.numpy()} ref {ref}")
    assert e_g <= (1e-9 if prec == "f64" else 8 * U32 * cond_s + 4e-3)
    assert e_a <= (1e-10 if prec == "f64" else 1e-3)


def test_c4_full_fp64_gradient_vs_finite_differences():
    dev = device()
    a = api()
    w = W.WORKLOADS["C4"]
    x, yv, om_np, om = _setup(w, "f64", dev)
    X = to_dev(x, torch.float32, dev)
    y = to_dev(yv, torch.float64, dev).reshape(-1, 1)
    th0 = np.log([w.ell, w.s, w.sigma2])

    def ll_at(th):
        h = a.Hyper(w.kernel, math.exp(th[0]), math.exp(th[1]))
        fw = a.forward(X, h, om, "f64", math.exp(th[2]), y, w.leaf_rows)
        return a.loglik(y, fw.sol.X, fw.sol.logdet, fw.sol.info, "f64").item(), fw

    note("C4 full fp64 gradient")
    ll0, fw = ll_at(th0)
    dth, _ = a.backward(X, a.Hyper(w.kernel, w.ell, w.s), om, "f64", fw.sol, fw.Q, w.sigma2, 0, fw.sol.X)
    g = dth.cpu().numpy()
    # central differences with one Richardson step: truncation O(h^4) is ~1e-8
    # here; rounding of the float64 log-likelihood (|ll| ~ 1e5, ~1e-14 relative)
    # divided by h gives ~1e-6 absolute.
    fd = np.zeros(3)
    h = 2e-3
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        d1 = (ll_at(th0 + h * e)[0] - ll_at(th0 - h * e)[0]) / (2 * h)
        d2 = (ll_at(th0 + 0.5 * h * e)[0] - ll_at(th0 - 0.5 * h * e)[0]) / h
        fd[k] = (4 * d2 - d1) / 3
    note(f"  ll {ll0:.10e} grad {g} fd {fd} diff {g - fd}")
    assert np.all(np.abs(g - fd) <= 1e-7 * np.abs(g) + 2e-9 * abs(ll0) / h)
