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
