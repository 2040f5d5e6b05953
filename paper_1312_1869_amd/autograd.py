"""torch.autograd.Function wrappers with the hand-written adjoint.

theta = (log ell, log s, log sigma2) is a float64 CPU tensor; points, Omega
and right-hand sides live on the GPU. Forward runs sketch -> blocked QR ->
Woodbury solve; backward calls lr_backward, which recomputes the derivative
kernel tiles (or reuses the fused forward's (dK/dlog ell) Omega).
"""
from __future__ import annotations

import dataclasses
import math

import torch

from . import api


@dataclasses.dataclass
class Config:
    kernel: str
    prec: str
    leaf_rows: int
    nu: float = 0.0
    fused: bool = False  # keep (dK/dlog ell) Omega from the forward sketch


def _hyper(theta: torch.Tensor, kernel: str):
    t = theta.detach().to("cpu", torch.float64).tolist()
    return api.Hyper(kernel, math.exp(t[0]), math.exp(t[1])), math.exp(t[2])


def _check_info(sol: api.SolveOut) -> None:
    info = int(sol.info.item())
    if info != 0:
        raise torch.linalg.LinAlgError(f"low-rank core factorisation failed (info = {info})")


class LowRankSolve(torch.autograd.Function):
    """X = K~(theta)^{-1} A."""

    @staticmethod
    def forward(ctx, theta, A, X, omega, cfg: Config):
        hyper, sigma2 = _hyper(theta, cfg.kernel)
        Ac = A.contiguous()
        fw = api.forward(X, hyper, omega, cfg.prec, sigma2, Ac, cfg.leaf_rows, nu=cfg.nu, want_yprime=cfg.fused)
        _check_info(fw.sol)
        ctx.save_for_backward(X, fw.Q, Ac, fw.R)
        ctx.fac = fw.sol
        ctx.yprime = fw.Yprime
        ctx.omega, ctx.cfg, ctx.hyper, ctx.sigma2 = omega, cfg, hyper, sigma2
        ctx.theta_dtype, ctx.theta_device = theta.dtype, theta.device
        return fw.sol.X

    @staticmethod
    def backward(ctx, gX):
        X, Q, A, R = ctx.saved_tensors
        dtheta, dA = api.backward(X, ctx.hyper, ctx.omega, ctx.cfg.prec, ctx.fac, Q, ctx.sigma2, 1, A,
                                  V=gX.contiguous().to(A.dtype), Yprime=ctx.yprime, want_dA=True, R=R,
                                  nu=ctx.cfg.nu)
        return dtheta.to(ctx.theta_device, ctx.theta_dtype), dA, None, None, None


class LowRankLogLik(torch.autograd.Function):
    """-1/2 y^T K~(theta)^{-1} y - 1/2 log|K~(theta)| (float64 scalar on the GPU)."""

    @staticmethod
    def forward(ctx, theta, y, X, omega, cfg: Config):
        hyper, sigma2 = _hyper(theta, cfg.kernel)
        yc = y.reshape(-1, 1).contiguous()
        fw = api.forward(X, hyper, omega, cfg.prec, sigma2, yc, cfg.leaf_rows, nu=cfg.nu, want_yprime=cfg.fused)
        _check_info(fw.sol)
        ll = api.loglik(yc, fw.sol.X, fw.sol.logdet, fw.sol.info, cfg.prec)
        ctx.save_for_backward(X, fw.Q, yc, fw.R)
        ctx.fac = fw.sol
        ctx.yprime = fw.Yprime
        ctx.omega, ctx.cfg, ctx.hyper, ctx.sigma2 = omega, cfg, hyper, sigma2
        ctx.theta_dtype, ctx.theta_device = theta.dtype, theta.device
        return ll.reshape(())

    @staticmethod
    def backward(ctx, g):
        X, Q, yc, R = ctx.saved_tensors
        dtheta, _ = api.backward(X, ctx.hyper, ctx.omega, ctx.cfg.prec, ctx.fac, Q, ctx.sigma2, 0, yc,
                                 Yprime=ctx.yprime, R=R, nu=ctx.cfg.nu)
        return (g.to(torch.float64) * dtheta).to(ctx.theta_device, ctx.theta_dtype), None, None, None, None
