"""Pins of the oracle's hyperparameter gradients."""
import numpy as np
import pytest

import workloads as W
from oracle import grad, lowrank


def _case(kind, n=512, d=24, leaf=128):
    w = W.small(W.WORKLOADS["C4"], n, d=d, leaf_rows=leaf).replace(kernel=kind)
    x = W.points(w)
    signs, cols = W.srht_draw(w)
    om = {"kind": "srht", "signs": signs, "cols": cols}
    return w, x, om


@pytest.mark.parametrize("kind", ["se", "matern32"])
def test_loglik_gradient_fd_and_dense(kind):
    w, x, om = _case(kind)
    yv = W.gp_targets(w, x)
    f = grad.forward(x, kind, w.ell, w.s, w.sigma2, om, yv.reshape(-1, 1), w.leaf_rows)
    alpha = f["X"][:, 0]
    g = grad.grad_loglik(x, kind, w.ell, w.s, w.sigma2, om, f["Q"], f, yv)
    gd, _ = grad.grad_loglik_dense(x, kind, w.ell, w.s, w.sigma2, om, yv)
    np.testing.assert_allclose(g, gd, rtol=1e-7)
    th = np.log([w.ell, w.s, w.sigma2])
    fd = grad.fd_gradient(lambda t: grad.loglik_at(t, x, kind, om, yv, w.leaf_rows), th)
    np.testing.assert_allclose(g, fd, rtol=2e-6)
    # Closed forms for log s and log sigma2.
    n, d = f["Q"].shape
    tr_kinv = (n - d) / w.sigma2 + np.trace(lowrank.s_solve(f["L"], np.eye(d)))
    ys = yv.astype(np.float64)
    assert g[1] == pytest.approx(alpha @ (ys - w.sigma2 * alpha) - (n - w.sigma2 * tr_kinv), rel=1e-9)
    assert g[2] == pytest.approx(0.5 * w.sigma2 * (alpha @ alpha - tr_kinv), rel=1e-9)


def test_solve_vjp_gradient_fd_and_dense():
    w, x, om = _case("se", n=256, d=20, leaf=64)
    rng = np.random.default_rng(11)
    a = rng.standard_normal((w.n, 3))
    abar = rng.standard_normal((w.n, 3))
    f = grad.forward(x, "se", w.ell, w.s, w.sigma2, om, a, w.leaf_rows)
    g, b = grad.grad_solve(x, "se", w.ell, w.s, w.sigma2, om, f["Q"], f, a, abar)
    gd, bd = grad.grad_solve_dense(x, "se", w.ell, w.s, w.sigma2, om, a, abar)
    np.testing.assert_allclose(g, gd, rtol=1e-7)
    np.testing.assert_allclose(b, bd, rtol=1e-8, atol=1e-8 * np.abs(bd).max())

    def obj(t):
        o = grad.forward(x, "se", np.exp(t[0]), np.exp(t[1]), np.exp(t[2]), om, a, w.leaf_rows)
        return float(np.sum(abar * o["X"]))

    fd = grad.fd_gradient(obj, np.log([w.ell, w.s, w.sigma2]))
    np.testing.assert_allclose(g, fd, rtol=2e-6)


@pytest.mark.parametrize("kind,nu_frac", [("se", 0.1), ("matern32", 0.5)])
def test_shifted_loglik_gradient_fd_and_dense(kind, nu_frac):
    """Shifted sketch Y = (K_f + nu I) Omega: the extra projector terms of the
    adjoint against the dense definition (with -nu P_Y) and finite differences
    of the shifted forward."""
    w, x, om = _case(kind)
    nu = nu_frac * w.sigma2
    yv = W.gp_targets(w, x)
    f = grad.forward(x, kind, w.ell, w.s, w.sigma2, om, yv.reshape(-1, 1), w.leaf_rows, nu=nu)
    g = grad.grad_loglik(x, kind, w.ell, w.s, w.sigma2, om, f["Q"], f, yv, nu=nu, r=f["R"])
    gd, _ = grad.grad_loglik_dense(x, kind, w.ell, w.s, w.sigma2, om, yv, nu=nu)
    np.testing.assert_allclose(g, gd, rtol=1e-7)
    th = np.log([w.ell, w.s, w.sigma2])
    fd = grad.fd_gradient(lambda t: grad.loglik_at(t, x, kind, om, yv, w.leaf_rows, nu=nu), th)
    np.testing.assert_allclose(g, fd, rtol=2e-6)
    # the shift changes the gradient (the extra terms are not vanishingly small)
    g0 = grad.grad_loglik(x, kind, w.ell, w.s, w.sigma2, om, f["Q"], f, yv)
    assert np.max(np.abs(g - g0) / np.abs(g)) > 1e-6


def test_shifted_solve_vjp_gradient_fd_and_dense():
    w, x, om = _case("se", n=256, d=20, leaf=64)
    nu = 0.3 * w.sigma2
    rng = np.random.default_rng(12)
    a = rng.standard_normal((w.n, 2))
    abar = rng.standard_normal((w.n, 2))
    f = grad.forward(x, "se", w.ell, w.s, w.sigma2, om, a, w.leaf_rows, nu=nu)
    g, b = grad.grad_solve(x, "se", w.ell, w.s, w.sigma2, om, f["Q"], f, a, abar, nu=nu, r=f["R"])
    gd, bd = grad.grad_solve_dense(x, "se", w.ell, w.s, w.sigma2, om, a, abar, nu=nu)
    np.testing.assert_allclose(g, gd, rtol=1e-7)
    np.testing.assert_allclose(b, bd, rtol=1e-8, atol=1e-8 * np.abs(bd).max())

    def obj(t):
        o = grad.forward(x, "se", np.exp(t[0]), np.exp(t[1]), np.exp(t[2]), om, a, w.leaf_rows, nu=nu)
        return float(np.sum(abar * o["X"]))

    fd = grad.fd_gradient(obj, np.log([w.ell, w.s, w.sigma2]))
    np.testing.assert_allclose(g, fd, rtol=2e-6)


def test_shifted_gaussian_omega_gradient_dense():
    """Gaussian Omega (Omega^T Omega != I) with a shift: the Omega^T Omega term."""
    w = W.small(W.WORKLOADS["C3"], 400, d=24, leaf_rows=100).replace(ell=0.3, sigma2=1e-2)
    x = W.points(w)
    om = {"kind": "gauss", "omega_t": W.gauss_omega(w).astype(np.float64)}
    nu = 0.2 * w.sigma2
    yv = W.rhs(w, m=1)[:, 0]
    f = grad.forward(x, w.kernel, w.ell, w.s, w.sigma2, om, yv.reshape(-1, 1), w.leaf_rows, nu=nu)
    g = grad.grad_loglik(x, w.kernel, w.ell, w.s, w.sigma2, om, f["Q"], f, yv, nu=nu, r=f["R"])
    gd, _ = grad.grad_loglik_dense(x, w.kernel, w.ell, w.s, w.sigma2, om, yv, nu=nu)
    np.testing.assert_allclose(g, gd, rtol=1e-7)
