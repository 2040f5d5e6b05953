"""Gradients with respect to (log ell, log s, log sigma2) (oracle).

Not in the paper: the hyperparameter adjoint of the approximation defined in
``oracle.lowrank`` (with nu = 0). For a scalar objective whose derivative with
respect to K_tilde is the symmetric matrix G, d/dtheta = tr(G dK_tilde/dtheta).

* log-likelihood: G = 1/2 (alpha alpha^T - K_tilde^{-1}), alpha = K_tilde^{-1} y.
* solve, with cotangent Abar of X = K_tilde^{-1} A: G = -1/2 (X B^T + B X^T),
  B = K_tilde^{-1} Abar, and dA = B.

With N = Y W^{-1} Y^T, Y = K_f Omega, W = Omega^T Y, Y' = (dK_f/dlog ell) Omega,
Phi = F^{-1} (so Y W^{-1} = Q Phi):

    d/dlog ell    = 2 <G Q Phi, Y'> - <Phi^T (Q^T G Q) Phi, Omega^T Y'>
    d/dlog s      = 2 tr(Q^T G Q C)            (N is proportional to s^2)
    d/dlog sigma2 = sigma2 tr(G)

The Q-basis projections of the solves use the Woodbury identity
Q^T K_tilde^{-1} = S^{-1} Q^T (Q has orthonormal columns in the method): for
the log-likelihood a = Q^T alpha is taken as S^{-1} Q^T y, so
G Q = 1/2 (alpha a^T - Q S^{-1}), Q^T G Q = 1/2 (a a^T - S^{-1}),
tr K_tilde^{-1} = (n - d) / sigma2 + tr S^{-1}; for the solve Q^T X = S^{-1}
Q^T A and Q^T B = S^{-1} Q^T Abar. The solves alpha, X, B themselves are the
forward's K_tilde^{-1} applied to y, A, Abar. Written this way the formulas
take Q, the core factors and Y' as given and never rely on Q^T Q = I holding
to more than the method's own arithmetic, so they can also be evaluated on
factors computed elsewhere (a reduced-precision Q promoted to float64).

With a shift nu > 0 the sketch is Y = (K_f + nu I) Omega and
K_tilde = sigma2 I + N - nu P_Y, P_Y = Q Q^T the projector onto range(Y)
(nu is a fixed method parameter, independent of theta). For a derivative
sketch Y'' = dY/dtheta, d P_Y = (I - P_Y) Y'' Y^+ + (Y^+)^T Y''^T (I - P_Y) with
Y^+ = R^{-1} Q^T, so every theta term gains
    - 2 nu <(G Q - Q Q^T G Q) R^{-T}, Y''>,
and the log s sketch is no longer proportional to Y: Y'' = 2 (Y - nu Omega).
Since (I - P_Y) Y = 0 and Q^T G Y = Q^T G Q R, the Y part of that sketch
still gives 2 tr(Q^T G Q C); the -2 nu Omega part adds
    -4 nu <G Q Phi, Omega> + 2 nu <Phi^T (Q^T G Q) Phi, Omega^T Omega>
    + 4 nu^2 <(G Q - Q Q^T G Q) R^{-T}, Omega>.
With nu = 0 all extra terms vanish.

``*_dense`` functions evaluate the same derivatives from the plain definition
with explicit n x n matrices (small n): dN = Y'' W^{-1} Y^T + Y W^{-1} Y''^T -
Y W^{-1} (Omega^T Y'') W^{-1} Y^T, and d P_Y from the pseudo-inverse formula.

Pins (tests/test_oracle_grad.py): central finite differences (Richardson
extrapolated) of the oracle's own forward, with and without a shift; the
dense product-rule form; the closed forms (nu = 0)
d/dlog s = alpha^T (y - sigma2 alpha) - (n - sigma2 tr K_tilde^{-1}) and
d/dlog sigma2 = sigma2/2 (alpha^T alpha - tr K_tilde^{-1}).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import kernels, lowrank, qr, sketch


def _phi(core: dict) -> np.ndarray:
    d = core["F"].shape[0] if "F" in core else core["C"].shape[0]
    return sla.lu_solve(core["lu"], np.eye(d), check_finite=False)


def _theta_terms(q, core, omega, yprime, gq, qgq, trace_g, sigma2, trace_scale, nu=0.0, r=None):
    phi = _phi(core)
    e = sketch.omega_t_apply(omega, yprime)
    t1 = 2.0 * float(np.sum((gq @ phi) * yprime))
    t2 = float(np.sum((phi.T @ qgq @ phi) * e))
    d_s = 2.0 * float(np.sum(qgq * core["C"]))
    d_ell = t1 - t2
    if nu != 0.0:
        n, d = q.shape
        om = sketch.omega_rows(omega, np.arange(n))
        # (G Q - Q Q^T G Q) R^{-T}, n x d
        bp = sla.solve_triangular(np.asarray(r, dtype=np.float64), (gq - q @ qgq).T, lower=False,
                                  check_finite=False).T
        d_ell -= 2.0 * nu * float(np.sum(bp * yprime))
        d_s += (-4.0 * nu * float(np.sum((gq @ phi) * om))
                + 2.0 * nu * float(np.sum((phi.T @ qgq @ phi) * (om.T @ om)))
                + 4.0 * nu * nu * float(np.sum(bp * om)))
    grad = np.array([d_ell, d_s, sigma2 * trace_g])
    # magnitude of what each component sums (for rounding-error scales in tests)
    scale = np.array([abs(t1) + abs(t2), 2.0 * float(np.sum(np.abs(qgq * core["C"]))), sigma2 * trace_scale])
    return grad, scale


def _check_shift(nu, r):
    if nu != 0.0 and r is None:
        raise ValueError("a shifted sketch (nu != 0) needs the R factor")


def grad_loglik(x, kind, ell, s, sigma2, omega, q, core, y, yprime=None, parts=False, nu=0.0, r=None):
    """Gradient of the approximate log-likelihood.

    ``core`` holds the forward's factors (``lu`` of F, ``C``, ``L``); with a
    shift ``nu`` the R factor ``r`` of the shifted sketch is needed too. With
    ``parts`` also returns, per component, the sum of the magnitudes of the
    terms it adds up (|T1| + |T2| for log ell; for log s and log sigma2 the
    terms of their closed forms, alpha^T y, sigma2 alpha^T alpha, n,
    sigma2 tr K~^{-1}).
    """
    _check_shift(nu, r)
    q = np.asarray(q, dtype=np.float64)
    n, d = q.shape
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    if yprime is None:
        yprime = sketch.sketch(x, kind, ell, s, omega, deriv=True)
    alpha = lowrank.apply(q, core["L"], y.reshape(-1, 1), sigma2)[:, 0]
    a = lowrank.s_solve(core["L"], q.T @ y)
    s_inv = lowrank.s_solve(core["L"], np.eye(d))
    gq = 0.5 * (np.outer(alpha, a) - q @ s_inv)
    qgq = 0.5 * (np.outer(a, a) - s_inv)
    tr_kinv = (n - d) / sigma2 + float(np.trace(s_inv))
    aa = float(alpha @ alpha)
    trace_g = 0.5 * (aa - tr_kinv)
    g, scale = _theta_terms(q, core, omega, yprime, gq, qgq, trace_g, sigma2, 0.5 * (aa + tr_kinv), nu, r)
    ya = abs(float(y @ alpha))
    scale[1] = ya + sigma2 * aa + n + sigma2 * tr_kinv
    return (g, scale) if parts else g


def grad_solve(x, kind, ell, s, sigma2, omega, q, core, a, abar, yprime=None, parts=False, nu=0.0, r=None):
    """Gradient of <Abar, K_tilde^{-1} A> for the forward's right-hand side A.
    Returns (dtheta, dA), or (dtheta, dA, scale) with ``parts`` (scale as in
    grad_loglik). A shift ``nu`` needs the R factor ``r``."""
    _check_shift(nu, r)
    q = np.asarray(q, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    abar = np.asarray(abar, dtype=np.float64)
    xsol = lowrank.apply(q, core["L"], a, sigma2)
    b = lowrank.apply(q, core["L"], abar, sigma2)
    if yprime is None:
        yprime = sketch.sketch(x, kind, ell, s, omega, deriv=True)
    qx = lowrank.s_solve(core["L"], q.T @ a)
    qb = lowrank.s_solve(core["L"], q.T @ abar)
    gq = -0.5 * (xsol @ qb.T + b @ qx.T)
    qgq = -0.5 * (qx @ qb.T + qb @ qx.T)
    trace_g = -float(np.sum(xsol * b))
    g, scale = _theta_terms(q, core, omega, yprime, gq, qgq, trace_g, sigma2, float(np.sum(np.abs(xsol * b))),
                            nu, r)
    return (g, b, scale) if parts else (g, b)


# ---------------------------------------------------------------- dense definitions

def _dense_parts(x, kind, ell, s, sigma2, omega, nu=0.0):
    """K_tilde and its theta derivatives (log ell, log s) from the definition."""
    n = np.asarray(x).shape[0]
    om = sketch.omega_dense(omega, n)
    kf = kernels.kernel_matrix(kind, x, x, ell, s)
    kp = kernels.kernel_matrix_dlogell(kind, x, x, ell, s)
    y = (kf + nu * np.eye(n)) @ om
    w = om.T @ y
    winv_yt = np.linalg.solve(w, y.T)
    nmat = y @ winv_yt
    ypinv = np.linalg.solve(y.T @ y, y.T)   # Y^+
    proj = y @ ypinv
    kt = sigma2 * np.eye(n) + nmat - nu * proj

    def dk(ydd):
        dn = ydd @ winv_yt + winv_yt.T @ ydd.T - winv_yt.T @ (om.T @ ydd) @ winv_yt
        dp = (np.eye(n) - proj) @ ydd @ ypinv
        return dn - nu * (dp + dp.T)

    return kt, dk(kp @ om), dk(2.0 * kf @ om)


def grad_loglik_dense(x, kind, ell, s, sigma2, omega, yv, nu=0.0):
    kt, dk_ell, dk_s = _dense_parts(x, kind, ell, s, sigma2, omega, nu)
    n = kt.shape[0]
    kinv = np.linalg.inv(kt)
    alpha = kinv @ np.asarray(yv, dtype=np.float64).reshape(-1)
    g = 0.5 * (np.outer(alpha, alpha) - kinv)
    return np.array([np.sum(g * dk_ell), np.sum(g * dk_s), sigma2 * np.trace(g)]), n


def grad_solve_dense(x, kind, ell, s, sigma2, omega, a, abar, nu=0.0):
    kt, dk_ell, dk_s = _dense_parts(x, kind, ell, s, sigma2, omega, nu)
    xs = np.linalg.solve(kt, np.asarray(a, dtype=np.float64))
    b = np.linalg.solve(kt, np.asarray(abar, dtype=np.float64))
    g = -0.5 * (xs @ b.T + b @ xs.T)
    return np.array([np.sum(g * dk_ell), np.sum(g * dk_s), sigma2 * np.trace(g)]), b


# ---------------------------------------------------------------- forward used by FD

def forward(x, kind, ell, s, sigma2, omega, a, leaf_rows, nu=0.0, k_round=None):
    """Sketch -> blocked QR -> Woodbury solve. Returns dict(Y, Q, R, core..., X, logdet)."""
    y = sketch.sketch(x, kind, ell, s, omega, nu=nu, k_round=k_round)
    q, r = qr.tsqr(y, leaf_rows)
    out = lowrank.solve(q, r, omega, sigma2, a, nu)
    out.update({"Y": y, "Q": q, "R": r})
    return out


def loglik_at(theta, x, kind, omega, yv, leaf_rows, nu=0.0):
    """Approximate log-likelihood at theta = (log ell, log s, log sigma2)."""
    ell, s, sigma2 = np.exp(theta[0]), np.exp(theta[1]), np.exp(theta[2])
    out = forward(x, kind, ell, s, sigma2, omega, np.asarray(yv).reshape(-1, 1), leaf_rows, nu=nu)
    return lowrank.loglik(yv, out["X"][:, 0], out["logdet"])


def fd_gradient(fun, theta, h=1e-3):
    """Central differences with one Richardson step (error O(h^4))."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.zeros_like(theta)
    for k in range(theta.shape[0]):
        e = np.zeros_like(theta)
        e[k] = 1.0
        d1 = (fun(theta + h * e) - fun(theta - h * e)) / (2 * h)
        d2 = (fun(theta + 0.5 * h * e) - fun(theta - 0.5 * h * e)) / h
        g[k] = (4.0 * d2 - d1) / 3.0
    return g
