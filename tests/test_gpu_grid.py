"""GPU parity of the hyperparameter-grid sketch (lr_sketch_grid) and of the
log-likelihood grid built on it (the grids over the range parameter of
Sec. 5.2), against the oracle run separately at every grid point.

SRHT: one pass serves two kernels, with the points prescaled for ell = 1 and
each kernel's squared distance scaled by 1/ell_g^2, so every Y_g is held to
the single-kernel SRHT bar, 16 log2(n) u times c sum_j |K_ij|. A dense Omega
runs the single-kernel sketch per grid point, so its Y_g equal lr_sketch's
bit for bit.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import grad as og, kernels, lowrank as olr, sketch as osk

from gpu_common import U32, U64, api, device, log2n, note, omega_pair, qr_fp64, to_dev, torch

pytestmark = pytest.mark.gpu


def _grid(kind, n_theta):
    ells = np.linspace(0.08, 0.3, n_theta)
    ss = np.linspace(0.7, 1.6, n_theta)
    return [(kind, float(e), float(s)) for e, s in zip(ells, ss)]


@pytest.mark.parametrize("prec,u", [("f32", U32), ("f64", U64)])
@pytest.mark.parametrize("kind", ["se", "matern32"])
def test_srht_grid_against_oracle(prec, u, kind):
    dev = device()
    a = api()
    w = W.small(W.WORKLOADS["C2"], 8192, d=200)          # d = 200: a ragged column count
    x = W.points(w)
    om_np, om = omega_pair(w, prec, dev)
    grid = _grid(kind, 5)                                 # two passes of two and one of one
    hyps = [a.Hyper(k, e, s) for k, e, s in grid]
    note(f"srht grid {kind} {prec} n={w.n} d={w.d} G={len(grid)} nu=0.01")
    Y = a.sketch_grid(to_dev(x, torch.float32, dev), hyps, om, prec, nu=0.01)
    torch.cuda.synchronize()
    Y = Y.double().cpu().numpy()
    for g, (k, ell, s) in enumerate(grid):
        ref = osk.sketch(x, k, ell, s, om_np, nu=0.01)
        kf = kernels.kernel_matrix(k, x.astype(np.float64), x.astype(np.float64), ell, s)
        sc = np.abs(kf).sum(axis=1, keepdims=True) / math.sqrt(w.n) + 0.01
        err = (np.abs(Y[g] - ref) / sc).max()
        note(f"  g={g} ell={ell:.3f} s={s:.3f}: max err / scale {err:.2e}")
        assert err <= 16 * log2n(w.n) * u


def test_dense_grid_equals_single_sketches():
    dev = device()
    a = api()
    w = W.small(W.WORKLOADS["C3"], 3000, d=96)
    x = to_dev(W.points(w), torch.float32, dev)
    _, om = omega_pair(w, "bf16", dev)
    hyps = [a.Hyper("matern32", e, s) for _, e, s in _grid("matern32", 3)]
    note(f"dense grid bf16 n={w.n} d={w.d} G=3")
    Y = a.sketch_grid(x, hyps, om, "bf16")
    for g, h in enumerate(hyps):
        y1, _ = a.sketch(x, h, om, "bf16")
        torch.cuda.synchronize()
        assert torch.equal(Y[g], y1)


def test_loglik_grid_fp64_against_oracle():
    """Log-likelihood at a 4-point grid over (ell, s, sigma2) in FP64 against the
    oracle's forward at each point: 1e-10 relative, plus four times the spread
    between the oracle with its own tree QR and with LAPACK's QR (the method's
    float64 sensitivity where d reaches the kernel's numerical rank)."""
    dev = device()
    a = api()
    w = W.small(W.WORKLOADS["C4"], 4096, d=64, leaf_rows=1024)
    x = W.points(w)
    yv = W.gp_targets(w, x)
    om_np, om = omega_pair(w, "f64", dev)
    grid = [(0.15, 1.2, 5e-3), (0.25, 1.5, 1e-2), (0.35, 1.0, 2e-2), (0.5, 2.0, 1e-2)]
    hyps = [a.Hyper("se", e, s) for e, s, _ in grid]
    note(f"loglik grid fp64 n={w.n} d={w.d} G={len(grid)}")
    ll = a.loglik_grid(to_dev(x, torch.float32, dev), hyps, [s2 for _, _, s2 in grid], om, "f64",
                       to_dev(yv, torch.float64, dev), w.leaf_rows).cpu().numpy()
    for g, (ell, s, s2) in enumerate(grid):
        ref = og.loglik_at(np.log([ell, s, s2]), x, "se", om_np, yv, w.leaf_rows)
        # near the kernel's numerical rank (ell = 0.5 here) two float64 QRs of
        # the same sketch already differ by more than 1e-10: the bar includes
        # the oracle's spread between its tree QR and LAPACK's QR
        yk = osk.sketch(x, "se", ell, s, om_np)
        q, r = qr_fp64(yk)
        core = olr.solve(q, r, om_np, s2, yv.reshape(-1, 1))
        ll_lap = olr.loglik(yv, core["X"][:, 0], core["logdet"])
        bar = 1e-10 * abs(ref) + 4.0 * abs(ref - ll_lap)
        note(f"  ell={ell} s={s} sigma2={s2}: {ll[g]:.12e} oracle {ref:.12e} (LAPACK-QR oracle {ll_lap:.12e})")
        assert abs(ll[g] - ref) <= bar
