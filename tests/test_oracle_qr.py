"""Pins of the oracle's Householder QR and blocked tree QR (Sec. 3.3, Eq. 1-4)."""
import numpy as np
import pytest

from oracle import qr


def _sign_norm_r(a):
    r = np.linalg.qr(a, mode="r")
    return r * np.where(np.diag(r) < 0, -1.0, 1.0)[:, None]


def test_householder_against_lapack():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((200, 37))
    v, tau, r = qr.householder_qr(a)
    assert np.all(np.tril(r, -1) == 0.0)
    q = qr.thin_q(v, tau)
    np.testing.assert_allclose(q @ r, a, atol=1e-13)
    np.testing.assert_allclose(q.T @ q, np.eye(37), atol=1e-14)
    s = np.where(np.diag(r) < 0, -1.0, 1.0)
    np.testing.assert_allclose(r * s[:, None], _sign_norm_r(a), rtol=1e-12, atol=1e-12)
    # The LAPACK convention gives beta = -sign(alpha) ||x|| for the first column.
    assert r[0, 0] == pytest.approx(-np.sign(a[0, 0]) * np.linalg.norm(a[:, 0]), rel=1e-14)


def test_householder_zero_column_gives_tau_zero():
    a = np.zeros((6, 3))
    a[:, 1] = [1, 2, 3, 4, 5, 6]
    v, tau, r = qr.householder_qr(a)
    assert tau[0] == 0.0 and r[0, 0] == 0.0
    np.testing.assert_allclose(qr.thin_q(v, tau) @ r, a, atol=1e-14)
    # x below alpha is zero but alpha is not: H = I, beta = alpha.
    b = np.eye(4)[:, :2] * 3.0
    v, tau, r = qr.householder_qr(b)
    assert tau[0] == 0.0 and r[0, 0] == 3.0


@pytest.mark.parametrize("n,d,leaf", [(1024, 16, 128), (1000, 20, 96), (777, 7, 7), (512, 32, 512)])
def test_tsqr_matches_plain_qr(n, d, leaf):
    rng = np.random.default_rng(n + d)
    y = rng.standard_normal((n, d)) @ np.diag(np.logspace(0, -6, d))
    q, r = qr.tsqr(y, leaf)
    assert np.all(np.tril(r, -1) == 0.0) and np.all(np.diag(r) >= 0)
    np.testing.assert_allclose(q @ r, y, atol=1e-14 * np.abs(y).max() * 10)
    np.testing.assert_allclose(q.T @ q, np.eye(d), atol=1e-13)
    np.testing.assert_allclose(r, _sign_norm_r(y), rtol=1e-10, atol=1e-14)


def test_tsqr_one_leaf_is_plain_householder():
    rng = np.random.default_rng(3)
    y = rng.standard_normal((300, 12))
    q, r = qr.tsqr(y, 300, normalize_signs=False)
    v, tau, r0 = qr.householder_qr(y)
    np.testing.assert_array_equal(r, r0)
    np.testing.assert_array_equal(q, qr.thin_q(v, tau))


def test_tsqr_tree_shape_invariance():
    rng = np.random.default_rng(4)
    y = rng.standard_normal((4096, 24))
    rs = [qr.tsqr(y, leaf)[1] for leaf in (4096, 1024, 500, 96, 32)]
    for r in rs[1:]:
        np.testing.assert_allclose(r, rs[0], rtol=1e-11, atol=1e-12)


def test_leaf_shape_errors():
    with pytest.raises(ValueError):
        qr.leaf_bounds(100, 8, 16)
    with pytest.raises(ValueError):
        qr.leaf_bounds(100, 48, 16)  # last block has 4 < 16 rows
    assert qr.leaf_bounds(100, 42, 16) == [(0, 42), (42, 84), (84, 100)]


@pytest.mark.parametrize("group", [1, 2, 4, 8])
def test_grouped_sequential_scheme_matches_lapack(group):
    rng = np.random.default_rng(group)
    n, d, leaf = 8 * 40, 12, 40
    a = rng.standard_normal((n, d)) @ np.diag(np.logspace(0, -6, d))
    q, r = qr.tsqr_grouped(a, leaf, group)
    q_ref, r_ref = np.linalg.qr(a)
    sg = np.where(np.diag(r_ref) < 0, -1.0, 1.0)
    np.testing.assert_allclose(r, r_ref * sg[:, None], rtol=0, atol=1e-12 * np.abs(r_ref).max())
    np.testing.assert_allclose(q, q_ref * sg[None, :], rtol=0, atol=1e-9)
    np.testing.assert_allclose(q @ r, a, rtol=0, atol=1e-13 * np.abs(a).max())
    assert np.all(np.tril(r, -1) == 0.0) and np.all(np.diag(r) >= 0)
    if group == 1:
        q1, r1 = qr.tsqr(a, leaf)
        np.testing.assert_allclose(r, r1, rtol=0, atol=1e-14 * np.abs(r1).max())


def test_grouped_scheme_needs_whole_groups():
    with pytest.raises(ValueError):
        qr.tsqr_grouped(np.ones((300, 4)), 100, 2)
