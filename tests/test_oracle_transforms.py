"""Pins of the oracle's discrete cosine / Hartley structured Omega (Sec. 3.2,
Def. 1 with T the DCT-II or the discrete Hartley transform; Sec. 5, Table 3)."""
import numpy as np
import pytest
import scipy.fft

import workloads as W
from oracle import grad, kernels, lowrank, sketch, transforms


def _draw(n, d, seed=0):
    g = np.random.default_rng(seed)
    signs = (g.integers(0, 2, n) * 2 - 1).astype(np.int8)
    cols = np.sort(g.choice(n, d, replace=False)).astype(np.int32)
    return signs, cols


@pytest.mark.parametrize("n", [1, 5, 12, 64, 100])
def test_dct_entries_match_scipy(n):
    # scipy's orthonormal DCT-II of the identity's columns gives T^T
    t_ref = scipy.fft.dct(np.eye(n), type=2, norm="ortho", axis=0).T
    t = transforms.transform_entries("dct", n, np.arange(n), np.arange(n))
    np.testing.assert_allclose(t, t_ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [1, 7, 16, 90])
def test_dht_entries_match_fft(n):
    f = scipy.fft.fft(np.eye(n), axis=0)
    t_ref = (f.real - f.imag) / np.sqrt(n)
    t = transforms.transform_entries("dht", n, np.arange(n), np.arange(n))
    np.testing.assert_allclose(t, t_ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("kind", transforms.KINDS)
@pytest.mark.parametrize("n", [50, 257])
def test_transform_is_orthogonal_and_omega_orthonormal(kind, n):
    t = transforms.transform_entries(kind, n, np.arange(n), np.arange(n))
    np.testing.assert_allclose(t.T @ t, np.eye(n), rtol=0, atol=1e-12)
    signs, cols = _draw(n, 19, seed=n)
    om = transforms.omega_dense(kind, signs, cols)
    np.testing.assert_allclose(om.T @ om, np.eye(19), rtol=0, atol=1e-13)


def test_dht_is_its_own_inverse_and_dct_of_constant():
    n = 48
    h = transforms.transform_entries("dht", n, np.arange(n), np.arange(n))
    np.testing.assert_allclose(h, h.T, rtol=0, atol=1e-15)
    np.testing.assert_allclose(h @ h, np.eye(n), rtol=0, atol=1e-12)
    c = transforms.transform_entries("dct", n, np.arange(n), np.arange(n))
    e0 = np.zeros(n)
    e0[0] = np.sqrt(n)
    np.testing.assert_allclose(c.T @ np.ones(n), e0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", transforms.KINDS)
def test_angle_reduction_matches_unreduced_angle(kind):
    # large indices: the reduced form must agree with the plain float64 angle
    # to the plain angle's own rounding (~|angle| * 2^-53)
    n = 100003
    rows = np.array([0, 1, 4999, 77777, n - 1])
    cols = np.array([0, 3, 12345, 99999, n - 2])
    t = transforms.transform_entries(kind, n, rows, cols)
    j, p = rows[:, None].astype(np.float64), cols[None, :].astype(np.float64)
    if kind == "dct":
        ang = np.pi * (2 * j + 1) * p / (2 * n)
        ref = np.where(p == 0, np.sqrt(1.0 / n), np.sqrt(2.0 / n)) * np.cos(ang)
    else:
        ang = 2 * np.pi * j * p / n
        ref = (np.cos(ang) + np.sin(ang)) / np.sqrt(n)
    assert np.all(np.abs(t - ref) <= 4 * np.abs(ang) * 2.0 ** -53 / np.sqrt(n) + 1e-18)


@pytest.mark.parametrize("kind", transforms.KINDS)
@pytest.mark.parametrize("n", [96, 131])
def test_fast_applies_match_dense(kind, n):
    signs, cols = _draw(n, 13, seed=3)
    om = transforms.omega_dense(kind, signs, cols)
    m = np.random.default_rng(1).standard_normal((5, n))
    np.testing.assert_allclose(transforms.right_apply(m, kind, signs, cols), m @ om, rtol=0, atol=1e-12)
    q = np.random.default_rng(2).standard_normal((n, 7))
    np.testing.assert_allclose(transforms.left_apply_t(q, kind, signs, cols), om.T @ q, rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", transforms.KINDS)
def test_sketch_with_structured_omega_matches_dense_product(kind):
    n, d = 300, 16
    x = np.random.default_rng(5).random((n, 2)).astype(np.float32)
    signs, cols = _draw(n, d, seed=9)
    om = {"kind": kind, "signs": signs, "cols": cols}
    y = sketch.sketch(x, "se", 0.3, 1.2, om, nu=0.01)
    kf = kernels.kernel_matrix("se", x.astype(np.float64), x.astype(np.float64), 0.3, 1.2)
    dense = transforms.omega_dense(kind, signs, cols)
    np.testing.assert_allclose(y, (kf + 0.01 * np.eye(n)) @ dense, rtol=0, atol=1e-12)
    np.testing.assert_allclose(sketch.omega_rows(om, np.array([0, 17, n - 1])), dense[[0, 17, n - 1]],
                               rtol=0, atol=0)


@pytest.mark.parametrize("kind", transforms.KINDS)
def test_method_with_structured_omega_matches_dense_definition(kind):
    # the Woodbury form in the Q basis against (sigma2 I + Y W^-1 Y^T)^-1 A, and
    # an exact-rank signal reproduced: n not a power of two
    w = W.small(W.WORKLOADS["C1"], 300, d=24, leaf_rows=100)
    x = W.points(w)
    a = W.rhs(w, m=3)
    signs, cols = W.srht_draw(w)
    om = {"kind": kind, "signs": signs, "cols": cols}
    sigma2 = 1e-2
    f = grad.forward(x, "se", 0.3, 1.0, sigma2, om, a, w.leaf_rows)
    x_dense, ld_dense, sign = lowrank.solve_dense(f["Y"], sketch.omega_dense(om, w.n), sigma2, a)
    assert f["info"] == 0 and sign > 0
    np.testing.assert_allclose(f["X"], x_dense, rtol=1e-8, atol=1e-8 * np.abs(x_dense).max())
    assert abs(f["logdet"] - ld_dense) <= 1e-9 * abs(ld_dense)
    # exact rank: K_f = B B^T with rank 10 < d is reproduced to round-off
    b = np.random.default_rng(4).standard_normal((w.n, 10))
    kf = b @ b.T
    y = kf @ sketch.omega_dense(om, w.n)
    from oracle import qr
    q, r = qr.tsqr(y, w.leaf_rows)
    out = lowrank.solve(q, r, om, sigma2, a)
    x_true = np.linalg.solve(kf + sigma2 * np.eye(w.n), a)
    np.testing.assert_allclose(out["X"], x_true, rtol=0, atol=1e-6 * np.abs(x_true).max())


def test_cos_pi_ratio_quadrants_and_exact_zeros():
    big_n = 12
    k = np.arange(-30, 31)
    np.testing.assert_allclose(transforms.cos_pi_ratio(k, big_n), np.cos(np.pi * k / big_n), rtol=0, atol=4e-15)
    assert np.all(transforms.cos_pi_ratio(np.array([6, 18, -6, 30]), big_n) == 0.0)
    # the cosine / Hartley zeros of the transforms are exact
    n = 8
    assert transforms.transform_entries("dht", n, np.array([3]), np.array([1]))[0, 0] == 0.0  # cas(3 pi / 4)
    assert transforms.transform_entries("dct", 2, np.array([0]), np.array([2]))[0, 0] == 0.0  # cos(pi / 2)
