"""Pins of the oracle's sketch Y = (K_f + nu I) Omega (Sec. 3.1-3.2)."""
import math

import numpy as np
import pytest
from scipy.linalg import hadamard
from scipy.spatial.distance import cdist

import workloads as W
from oracle import kernels, sketch


def _kf(x, kind, ell, s):
    r = cdist(x.astype(np.float64), x.astype(np.float64))
    if kind == "se":
        return s * s * np.exp(-0.5 * (r / ell) ** 2)
    u = math.sqrt(3.0) * r / ell
    return s * s * (1 + u) * np.exp(-u)


@pytest.mark.parametrize("kind", ["se", "matern32"])
def test_srht_sketch_equals_dense_product(kind):
    w = W.small(W.WORKLOADS["C1"], 1024, d=48).replace(kernel=kind)
    x = W.points(w)
    signs, cols = W.srht_draw(w)
    om = {"kind": "srht", "signs": signs, "cols": cols}
    dense = signs[:, None].astype(np.float64) * hadamard(w.n)[:, cols] / math.sqrt(w.n)
    y = sketch.sketch(x, kind, w.ell, w.s, om)
    np.testing.assert_allclose(y, _kf(x, kind, w.ell, w.s) @ dense, rtol=1e-11, atol=1e-12)
    nu = 0.3
    y_nu = sketch.sketch(x, kind, w.ell, w.s, om, nu=nu)
    np.testing.assert_allclose(y_nu, (_kf(x, kind, w.ell, w.s) + nu * np.eye(w.n)) @ dense,
                               rtol=1e-11, atol=1e-12)


def test_gauss_sketch_equals_dense_product_and_rows():
    w = W.small(W.WORKLOADS["C3"], 1500, d=70)
    x = W.points(w)
    om_t = W.gauss_omega(w)
    om = {"kind": "gauss", "omega_t": om_t}
    y = sketch.sketch(x, w.kernel, w.ell, w.s, om)
    ref = _kf(x, w.kernel, w.ell, w.s) @ om_t.T.astype(np.float64)
    np.testing.assert_allclose(y, ref, rtol=1e-11, atol=1e-11)
    rows = np.array([1499, 0, 700, 3])
    np.testing.assert_allclose(sketch.sketch_rows(x, rows, w.kernel, w.ell, w.s, om), y[rows], rtol=1e-12, atol=1e-14)


def test_sketch_linear_in_omega():
    w = W.small(W.WORKLOADS["C3"], 600, d=20)
    x = W.points(w)
    rng = np.random.default_rng(9)
    o1 = rng.standard_normal((20, 600))
    o2 = rng.standard_normal((20, 600))
    y1 = sketch.sketch(x, w.kernel, w.ell, w.s, {"kind": "gauss", "omega_t": o1})
    y2 = sketch.sketch(x, w.kernel, w.ell, w.s, {"kind": "gauss", "omega_t": o2})
    y12 = sketch.sketch(x, w.kernel, w.ell, w.s, {"kind": "gauss", "omega_t": 2 * o1 - o2})
    np.testing.assert_allclose(y12, 2 * y1 - y2, rtol=1e-12, atol=1e-12)


def test_bf16_rounding_grid():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.14159, 1e-3])
    r = sketch.round_to_bf16(v)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7 and goes to the even mantissa (1).
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7
    bits = W.bf16_bits(v.astype(np.float32))
    np.testing.assert_array_equal(W.bf16_to_f32(bits).astype(np.float64), r)


def test_bf16x2_split_error_bound_and_sketch():
    """bfloat16 keeps 8 significant bits (unit roundoff u = 2^-8): k_hi = bf16(k)
    is within u |k|, and k_lo = bf16(k - k_hi) within u of that remainder, so
    |k_hi + k_lo - k| <= u^2 |k| = 2^-16 |k|; the error reaches the 2^-17
    neighbourhood (the split is not exact), and the bf16x2 sketch is the plain
    product of the split entries with Omega."""
    rng = np.random.default_rng(8)
    v = rng.standard_normal(200000) * np.exp(rng.uniform(-20, 5, 200000))
    r2 = sketch.round_to_bf16x2(v)
    rel = np.abs(r2 - v) / np.abs(v)
    assert rel.max() <= 2.0 ** -16
    assert rel.max() >= 2.0 ** -18
    # one bf16 term alone is far coarser
    assert (np.abs(sketch.round_to_bf16(v) - v) / np.abs(v)).max() >= 2.0 ** -10
    w = W.small(W.WORKLOADS["C3"], 300, d=12)
    x = W.points(w)
    om = {"kind": "gauss", "omega_t": W.gauss_omega(w, round_bf16=True).astype(np.float64)}
    k = kernels.kernel_matrix(w.kernel, x, x, w.ell, w.s)
    hi = sketch.round_to_bf16(k)
    lo = sketch.round_to_bf16(k - hi)
    ref = (hi + lo) @ om["omega_t"].T
    np.testing.assert_allclose(sketch.sketch(x, w.kernel, w.ell, w.s, om, k_round="bf16x2"), ref, rtol=1e-13,
                               atol=1e-13 * np.abs(ref).max())
