"""GPU parity of lr_sketch against the oracle's Y = (K_f + nu I) Omega.

Error measure: the rounding error of a sum of n products is bounded by a
multiple of the sum of their absolute values, so every entry is compared
against the oracle relative to that scale:
  SRHT:  scale_i  = c sum_j |K_f[i, j]|        (row-wise)
  dense: scale_ik = sum_j |K_f[i, j]| |Omega[j, k]|
Tolerances are stated as multiples of the unit roundoff of the arithmetic
(kernel values take a few ulps, the transform/accumulation log2(n) or sqrt(n)
more); for bf16 the K entries themselves are rounded (2^-8 relative).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import kernels, sketch as osk

from gpu_common import U32, U64, api, device, hyper, log2n, note, omega_pair, to_dev, torch

pytestmark = pytest.mark.gpu


def _scale_srht(x, rows, w, n):
    k = kernels.kernel_matrix(w.kernel, np.asarray(x)[rows], x, w.ell, w.s)
    return np.abs(k).sum(axis=1, keepdims=True) / math.sqrt(n)


def _scale_dense(x, rows, w, om_t):
    k = kernels.kernel_matrix(w.kernel, np.asarray(x)[rows], x, w.ell, w.s)
    return np.abs(k) @ np.abs(om_t.astype(np.float64)).T


def _bf16_ambiguity(x, rows, w, om_t, deriv=False):
    """Sum over j of |Omega_jk| times one bf16 spacing of K[i, j], taken over the
    entries whose float64 value lies within the float32 evaluation error of a
    bf16 rounding midpoint: only those may round to the other neighbour on the
    GPU (which rounds its float32 value). Everything else must agree to within
    float32 accumulation error."""
    kf = kernels.kernel_matrix_dlogell if deriv else kernels.kernel_matrix
    k = np.abs(kf(w.kernel, np.asarray(x)[rows], x, w.ell, w.s))
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(k > 0, k, 1.0)))
    spacing = np.exp2(e - 7)
    r = osk.round_to_bf16(k)
    to_mid = 0.5 * spacing - np.abs(k - r)
    delta = 16 * U32 * (1.0 + np.abs(e)) * k
    amb = np.where((k > 0) & (to_mid <= delta), spacing, 0.0)
    return amb @ np.abs(om_t.astype(np.float64)).T


def _run(w, prec, dev, want_yprime=False, nu=0.0, n=None, d=None):
    a = api()
    n = w.n if n is None else n
    x = W.points(w, n)
    om_np, om = omega_pair(w, prec, dev, n, d)
    X = to_dev(x, torch.float32, dev)
    note(f"sketch {w.name} n={n} d={om.d} prec={prec} yprime={want_yprime} nu={nu}")
    Y, Yp = a.sketch(X, hyper(w), om, prec, nu=nu, want_yprime=want_yprime)
    torch.cuda.synchronize()
    return x, om_np, (None if Y is None else Y.cpu().double().numpy()), (None if Yp is None else Yp.cpu().double().numpy())


@pytest.mark.parametrize("prec,tol_u", [("f64", U64), ("f32", U32)])
def test_srht_c1_full(prec, tol_u):
    dev = device()
    w = W.WORKLOADS["C1"]
    x, om, y, _ = _run(w, prec, dev)
    ref = osk.sketch(x, w.kernel, w.ell, w.s, om)
    sc = _scale_srht(x, np.arange(w.n), w, w.n)
    err = np.abs(y - ref) / sc
    note(f"  max err / (c |k_i|_1) = {err.max():.3e}  (u = {tol_u:.1e})")
    assert err.max() <= 16 * log2n(w.n) * tol_u


@pytest.mark.parametrize("kind", ["se", "matern32"])
def test_srht_ragged_d_and_derivative_f32(kind):
    dev = device()
    w = W.small(W.WORKLOADS["C2"], 8192, d=200).replace(kernel=kind)
    x, om, y, yp = _run(w, "f32", dev, want_yprime=True)
    ref = osk.sketch(x, w.kernel, w.ell, w.s, om)
    refd = osk.sketch(x, w.kernel, w.ell, w.s, om, deriv=True)
    sc = _scale_srht(x, np.arange(w.n), w, w.n)
    e1 = (np.abs(y - ref) / sc).max()
    e2 = (np.abs(yp - refd) / (sc * 4.0)).max()  # dk/dlog ell <= 4 max k for these kernels
    note(f"  Y err {e1:.3e}  Y' err {e2:.3e}")
    assert e1 <= 16 * log2n(w.n) * U32
    assert e2 <= 16 * log2n(w.n) * U32


def test_srht_small_n_below_chunk_and_nu():
    dev = device()
    w = W.small(W.WORKLOADS["C1"], 256, d=17)
    x, om, y, _ = _run(w, "f64", dev, nu=0.37)
    ref = osk.sketch(x, w.kernel, w.ell, w.s, om, nu=0.37)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_srht_c2_full_sampled_rows():
    dev = device()
    w = W.WORKLOADS["C2"]
    x, om, y, _ = _run(w, "f32", dev)
    rows = np.random.default_rng(0).choice(w.n, 48, replace=False)
    ref = osk.sketch_rows(x, rows, w.kernel, w.ell, w.s, om)
    err = (np.abs(y[rows] - ref) / _scale_srht(x, rows, w, w.n)).max()
    note(f"  C2 sampled err {err:.3e}")
    assert err <= 16 * log2n(w.n) * U32


def test_srht_c5_full_fused_sampled_rows():
    dev = device()
    w = W.WORKLOADS["C5"]
    x, om, y, yp = _run(w, "f32", dev, want_yprime=True)
    rows = np.random.default_rng(1).choice(w.n, 12, replace=False)
    ref = osk.sketch_rows(x, rows, w.kernel, w.ell, w.s, om)
    refd = osk.sketch_rows(x, rows, w.kernel, w.ell, w.s, om, deriv=True)
    sc = _scale_srht(x, rows, w, w.n)
    e1 = (np.abs(y[rows] - ref) / sc).max()
    e2 = (np.abs(yp[rows] - refd) / (4 * sc)).max()
    note(f"  C5 sampled err Y {e1:.3e} Y' {e2:.3e}")
    assert e1 <= 16 * log2n(w.n) * U32
    assert e2 <= 16 * log2n(w.n) * U32


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("kind", ["matern32", "se"])
def test_dense_ragged(prec, kind):
    dev = device()
    w = W.small(W.WORKLOADS["C3"], 3000, d=100).replace(kernel=kind, ell=0.2)
    x, om, y, _ = _run(w, prec, dev)
    om_t = om["omega_t"]
    sc = _scale_dense(x, np.arange(w.n), w, om_t)
    if prec == "bf16":
        ref = osk.sketch(x, w.kernel, w.ell, w.s, om, k_round="bf16")
        amb = _bf16_ambiguity(x, np.arange(w.n), w, om_t)
        excess = (np.abs(y - ref) - amb) / sc
        note(f"  bf16 vs bf16-rounded oracle: max err {(np.abs(y - ref) / sc).max():.3e}, "
             f"beyond rounding ambiguity {excess.max():.3e}")
        assert excess.max() <= 4 * math.sqrt(w.n) * U32
        exact = osk.sketch(x, w.kernel, w.ell, w.s, om)
        err2 = (np.abs(y - exact) / sc).max()
        note(f"  bf16 vs exact oracle {err2:.3e} (K rounding 2^-9 = {2**-9:.2e})")
        assert err2 <= 2.0 ** -8
    else:
        u = U64 if prec == "f64" else U32
        ref = osk.sketch(x, w.kernel, w.ell, w.s, om)
        err = (np.abs(y - ref) / sc).max()
        note(f"  {prec} err {err:.3e}")
        assert err <= 4 * math.sqrt(w.n) * u + 16 * u


@pytest.mark.parametrize("kind", ["matern32", "se"])
def test_dense_bf16x2(kind):
    """Two-term bf16 split of every kernel entry (k_hi + k_lo, 16 bits). The
    GPU splits its float32 value k32, the oracle its float64 value k; each
    split is within 2^-16 of what it splits, so the entries differ by at most
    2^-15 |k| plus the float32 evaluation error (16 u32 |k|), and the sums add
    the float32 accumulation error (4 sqrt(n) u32) of the scale."""
    dev = device()
    w = W.small(W.WORKLOADS["C3"], 3000, d=100).replace(kernel=kind, ell=0.2)
    x, om, y, yp = _run(w, "bf16x2", dev, want_yprime=True, nu=0.1)
    om_t = om["omega_t"]
    rows = np.arange(w.n)
    sc = _scale_dense(x, rows, w, om_t) + 0.1 * np.abs(om_t.T)
    ref = osk.sketch(x, w.kernel, w.ell, w.s, om, nu=0.1, k_round="bf16x2")
    refd = osk.sketch(x, w.kernel, w.ell, w.s, om, deriv=True, k_round="bf16x2")
    kd = np.abs(kernels.kernel_matrix_dlogell(w.kernel, x, x, w.ell, w.s))
    scd = kd @ np.abs(om_t.astype(np.float64)).T
    e1 = (np.abs(y - ref) / sc).max()
    e2 = (np.abs(yp - refd) / scd).max()
    exact = osk.sketch(x, w.kernel, w.ell, w.s, om, nu=0.1)
    e3 = (np.abs(y - exact) / sc).max()
    bar = 2.0 ** -15 + 16 * U32 + 4 * math.sqrt(w.n) * U32
    note(f"  bf16x2 vs bf16x2 oracle: Y {e1:.3e} Y' {e2:.3e} (bar {bar:.2e}); vs exact {e3:.3e}")
    assert e1 <= bar and e2 <= bar
    assert e3 <= 2.0 ** -16 + bar


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_dense_derivative_and_nu(prec):
    dev = device()
    w = W.small(W.WORKLOADS["C3"], 1100, d=40)
    x, om, y, yp = _run(w, prec, dev, want_yprime=True, nu=0.25)
    om_t = om["omega_t"]
    kr = "bf16" if prec == "bf16" else None
    ref = osk.sketch(x, w.kernel, w.ell, w.s, om, nu=0.25, k_round=kr)
    refd = osk.sketch(x, w.kernel, w.ell, w.s, om, deriv=True, k_round=kr)
    rows = np.arange(w.n)
    sc = _scale_dense(x, rows, w, om_t) + 0.25 * np.abs(om_t.T)
    kd = np.abs(kernels.kernel_matrix_dlogell(w.kernel, x, x, w.ell, w.s))
    scd = kd @ np.abs(om_t.astype(np.float64)).T
    amb = amb_d = 0.0
    if prec == "bf16":
        amb = _bf16_ambiguity(x, rows, w, om_t)
        amb_d = _bf16_ambiguity(x, rows, w, om_t, deriv=True)
    e1 = ((np.abs(y - ref) - amb) / sc).max()
    e2 = ((np.abs(yp - refd) - amb_d) / scd).max()
    note(f"  {prec}: Y {e1:.3e} Y' {e2:.3e} (beyond bf16 rounding ambiguity)")
    assert e1 <= 4 * math.sqrt(w.n) * U32 + 16 * U32
    assert e2 <= 4 * math.sqrt(w.n) * U32 + 16 * U32


def test_dense_c3_full_sampled_rows():
    dev = device()
    w = W.WORKLOADS["C3"]
    x, om, y, _ = _run(w, "bf16", dev)
    rows = np.concatenate([[0, w.n - 1], np.random.default_rng(2).choice(w.n, 30, replace=False)])
    ref = osk.sketch_rows(x, rows, w.kernel, w.ell, w.s, om, k_round="bf16")
    sc = _scale_dense(x, rows, w, om["omega_t"])
    amb = _bf16_ambiguity(x, rows, w, om["omega_t"])
    err = (np.abs(y[rows] - ref) / sc).max()
    excess = ((np.abs(y[rows] - ref) - amb) / sc).max()
    note(f"  C3 sampled bf16 err {err:.3e}, beyond rounding ambiguity {excess:.3e}")
    assert excess <= 4 * math.sqrt(w.n) * U32
