"""Pins of the oracle's Woodbury-form solve, log-determinant and core."""
import math

import numpy as np
import pytest
from scipy.linalg import hadamard
from scipy.stats import ortho_group

import workloads as W
from oracle import grad, kernels, lowrank, qr, sketch


def _srht(w):
    signs, cols = W.srht_draw(w)
    return {"kind": "srht", "signs": signs, "cols": cols}


def test_matches_dense_definition_c1_shape():
    w = W.WORKLOADS["C1"]
    x, a = W.points(w), W.rhs(w)
    om = _srht(w)
    out = grad.forward(x, w.kernel, w.ell, w.s, w.sigma2, om, a, w.leaf_rows)
    assert out["info"] == 0
    xd, ld, sign = lowrank.solve_dense(out["Y"], sketch.omega_dense(om, w.n), w.sigma2, a)
    assert sign > 0
    np.testing.assert_allclose(out["X"], xd, rtol=0, atol=1e-9 * np.abs(xd).max())
    assert out["logdet"] == pytest.approx(ld, rel=1e-12)


@pytest.mark.parametrize("nu", [0.0, 0.05])
def test_matches_dense_definition_gauss_with_shift(nu):
    w = W.small(W.WORKLOADS["C3"], 768, d=40, leaf_rows=128, m=3).replace(ell=0.3, sigma2=1e-1)
    x, a = W.points(w), W.rhs(w)
    om = {"kind": "gauss", "omega_t": W.gauss_omega(w, round_bf16=False)}
    out = grad.forward(x, w.kernel, w.ell, w.s, w.sigma2, om, a, w.leaf_rows, nu=nu)
    assert out["info"] == 0
    xd, ld, _ = lowrank.solve_dense(out["Y"], sketch.omega_dense(om, w.n), w.sigma2, a, nu=nu)
    np.testing.assert_allclose(out["X"], xd, rtol=0, atol=1e-8 * np.abs(xd).max())
    assert out["logdet"] == pytest.approx(ld, rel=1e-10)


def _exact_rank_case(rank, n=512, d=32, sigma2=1e-2):
    rng = np.random.default_rng(rank)
    phi = rng.standard_normal((n, rank))
    kf = phi @ phi.T
    om_t = rng.standard_normal((d, n)) / math.sqrt(d)
    y = kf @ om_t.T
    q, r = qr.tsqr(y, 128)
    a = rng.standard_normal((n, 2))
    return kf, om_t, q, r, a, sigma2


@pytest.mark.parametrize("rank", [32, 16, 5])
def test_exact_rank_recovers_true_inverse(rank):
    kf, om_t, q, r, a, sigma2 = _exact_rank_case(rank)
    out = lowrank.solve(q, r, {"kind": "gauss", "omega_t": om_t}, sigma2, a)
    k = kf + sigma2 * np.eye(kf.shape[0])
    ref = np.linalg.solve(k, a)
    cond = np.linalg.cond(k)
    np.testing.assert_allclose(out["X"], ref, atol=cond * 1e-14 * np.abs(ref).max())
    assert out["logdet"] == pytest.approx(np.linalg.slogdet(k)[1], rel=1e-8)


def test_full_dimension_sketch_is_exact():
    w = W.small(W.WORKLOADS["C1"], 256, d=256, leaf_rows=256, m=2).replace(ell=0.5, sigma2=0.5)
    x, a = W.points(w), W.rhs(w)
    om = _srht(w)
    out = grad.forward(x, w.kernel, w.ell, w.s, w.sigma2, om, a, w.leaf_rows)
    k = kernels.kernel_matrix(w.kernel, x, x, w.ell, w.s) + w.sigma2 * np.eye(w.n)
    np.testing.assert_allclose(out["X"], np.linalg.solve(k, a), rtol=1e-6, atol=1e-8)


def test_zero_signal_gives_a_over_sigma2():
    # Y = 0: every reflector has tau = 0, R = 0 and C = F^{-1} 0 = 0. (A Gaussian Omega
    # keeps F = Omega^T Q invertible; with the SRHT, F is the top block of Omega here.)
    w = W.small(W.WORKLOADS["C3"], 512, d=16, leaf_rows=64, m=3)
    x, a = W.points(w), W.rhs(w)
    om = {"kind": "gauss", "omega_t": W.gauss_omega(w, round_bf16=False)}
    out = grad.forward(x, w.kernel, w.ell, 0.0, 0.25, om, a, w.leaf_rows)
    assert out["info"] == 0
    np.testing.assert_allclose(out["X"], a / 0.25, rtol=1e-13)
    assert out["logdet"] == pytest.approx(w.n * math.log(0.25), rel=1e-13)


def test_invariant_under_omega_rotation():
    w = W.small(W.WORKLOADS["C3"], 600, d=24, leaf_rows=100, m=2).replace(ell=0.25, sigma2=1e-2)
    x, a = W.points(w), W.rhs(w)
    om_t = W.gauss_omega(w, round_bf16=False).astype(np.float64)
    t = ortho_group.rvs(24, random_state=7)
    o1 = grad.forward(x, w.kernel, w.ell, w.s, w.sigma2, {"kind": "gauss", "omega_t": om_t}, a, 100)
    o2 = grad.forward(x, w.kernel, w.ell, w.s, w.sigma2, {"kind": "gauss", "omega_t": t.T @ om_t}, a, 100)
    np.testing.assert_allclose(o1["X"], o2["X"], rtol=0, atol=1e-7 * np.abs(o1["X"]).max())
    assert o1["logdet"] == pytest.approx(o2["logdet"], rel=1e-10)


def test_cholesky_info_on_indefinite():
    s = np.diag([4.0, 1.0, -1.0, 2.0])
    lo, info = lowrank.cholesky_info(s)
    assert info == 3 and lo[1, 1] == 1.0
    spd = np.array([[4.0, 2.0], [2.0, 3.0]])
    lo, info = lowrank.cholesky_info(spd)
    assert info == 0
    np.testing.assert_allclose(lo @ lo.T, spd)
    np.testing.assert_allclose(lo, np.linalg.cholesky(spd))


def test_shift_beyond_spectrum_reports_not_pd():
    w = W.small(W.WORKLOADS["C1"], 256, d=16, leaf_rows=64)
    x, a = W.points(w), W.rhs(w)
    om = _srht(w)
    y = sketch.sketch(x, w.kernel, w.ell, w.s, om)
    q, r = qr.tsqr(y, w.leaf_rows)
    c = lowrank.core(q, r, om, w.sigma2, 0.0)
    lam_min = np.linalg.eigvalsh(c["C"]).min()
    bad = lowrank.core(q, r, om, w.sigma2, nu=w.sigma2 + lam_min + 1.0)
    assert bad["info"] > 0


def test_exact_dense_reference_c1_is_reproducible():
    """The stored exact-dense quantities of the plain FP64 workload
    (tests/golden/exact_dense_reference.txt, written by make_exact_reference.py)
    are reproduced here: the exact K^-1 A solves K X = A to round-off, and the
    method's X~ is a rank-64 approximation whose error against it (about 12%
    at sigma2 = 1e-4, Sec. 3.1) is a property of the method, not of a path."""
    from conftest import read_golden

    gold = {k: float(v) for k, v in read_golden("exact_dense_reference.txt")}
    w = W.WORKLOADS["C1"]
    x = W.points(w).astype(np.float64)
    a = W.rhs(w).astype(np.float64)
    k = kernels.kernel_matrix(w.kernel, x, x, w.ell, w.s) + w.sigma2 * np.eye(w.n)
    lo = np.linalg.cholesky(k)
    xe = np.linalg.solve(lo.T, np.linalg.solve(lo, a))
    assert np.linalg.norm(k @ xe - a) <= 1e-6 * np.linalg.norm(k) * np.linalg.norm(xe)
    assert abs(np.linalg.norm(xe) - gold["c1_x_exact_fro"]) <= 1e-8 * gold["c1_x_exact_fro"]
    ld = 2.0 * float(np.sum(np.log(np.diag(lo))))
    assert abs(ld - gold["c1_logdet_exact"]) <= 1e-10 * abs(ld)
    fwd = grad.forward(W.points(w), w.kernel, w.ell, w.s, w.sigma2, _srht(w), W.rhs(w), w.leaf_rows)
    err = np.linalg.norm(fwd["X"] - xe) / np.linalg.norm(xe)
    assert abs(err - gold["c1_method_x_relerr"]) <= 1e-6 * err
    assert 0.0 < err < 1.0


def test_psd_part_is_nearest_psd_and_idempotent():
    rng = np.random.default_rng(3)
    v = ortho_group.rvs(12, random_state=5)
    lam = np.array([5.0, 3.0, 2.0, 1.0, 0.5, 0.1, 0.0, -1e-3, -0.2, -1.0, -2.0, -4.0])
    b = (v * lam) @ v.T
    bp = lowrank.psd_part(b)
    np.testing.assert_allclose(bp, bp.T, rtol=0, atol=1e-14)
    assert np.linalg.eigvalsh(bp).min() >= -1e-13
    # distance to the PSD cone in the Frobenius norm = norm of the negative part
    np.testing.assert_allclose(np.linalg.norm(b - bp), np.linalg.norm(lam[lam < 0]), rtol=1e-12)
    # any other PSD matrix (here random ones) is no closer
    for _ in range(5):
        g = rng.standard_normal((12, 12))
        assert np.linalg.norm(b - g @ g.T) >= np.linalg.norm(b - bp)
    np.testing.assert_allclose(lowrank.psd_part(bp), bp, rtol=0, atol=1e-13)
    p = (v * np.abs(lam)) @ v.T
    np.testing.assert_allclose(lowrank.psd_part(p), p, rtol=0, atol=1e-13)


@pytest.mark.parametrize("clip", [False, True])
def test_projection_matches_dense_definition(clip):
    w = W.small(W.WORKLOADS["C1"], 256, d=24, leaf_rows=64)
    x = W.points(w).astype(np.float64)
    a = W.rhs(w, m=3)
    om = _srht(w)
    y = sketch.sketch(W.points(w), "se", 0.25, 1.1, om)
    q, r = qr.tsqr(y, w.leaf_rows)
    kf = kernels.kernel_matrix("se", x, x, 0.25, 1.1)
    kq = kf @ q
    sigma2 = 1e-2
    out = lowrank.projection_solve(q, kq, sigma2, a, clip=clip)
    kt = sigma2 * np.eye(w.n) + q @ (q.T @ kf @ q) @ q.T
    np.testing.assert_allclose(out["X"], np.linalg.solve(kt, a), rtol=1e-9, atol=1e-9 * np.abs(a).max() / sigma2)
    sign, ld = np.linalg.slogdet(kt)
    assert sign > 0 and abs(out["logdet"] - ld) <= 1e-10 * abs(ld)


def test_projection_exact_when_basis_holds_the_signal():
    # K_f of rank 8 and a basis whose first 8 columns span its range: K~ = K
    rng = np.random.default_rng(11)
    n, d = 200, 20
    b = rng.standard_normal((n, 8))
    kf = b @ b.T
    q, _ = np.linalg.qr(np.hstack([b, rng.standard_normal((n, d - 8))]))
    a = rng.standard_normal((n, 2))
    out = lowrank.projection_solve(q, kf @ q, 0.05, a)
    np.testing.assert_allclose(out["X"], np.linalg.solve(kf + 0.05 * np.eye(n), a), rtol=1e-9, atol=1e-9)
