"""Pins of the oracle's Walsh-Hadamard transform and SRHT (Def. 1, Sec. 3.2)."""
import numpy as np
import pytest
from scipy.linalg import hadamard

from oracle import srht


@pytest.mark.parametrize("n", [1, 2, 8, 64, 1024])
def test_sylvester_matches_scipy(n):
    np.testing.assert_array_equal(srht.hadamard_sylvester(n), hadamard(n))


@pytest.mark.parametrize("n", [2, 16, 512, 4096])
def test_fwht_matches_matrix_and_is_involution(n):
    rng = np.random.default_rng(n)
    v = rng.standard_normal((3, n))
    t = srht.fwht(v, axis=1)
    np.testing.assert_allclose(t, v @ hadamard(n).T, rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(srht.fwht(t, axis=1), n * v, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(srht.fwht(v.T, axis=0), t.T, rtol=1e-14, atol=1e-12)


def test_not_pow2_rejected():
    with pytest.raises(ValueError):
        srht.fwht(np.ones(12))
    with pytest.raises(ValueError):
        srht.hadamard_sylvester(12)


def _draw(n, d, seed):
    rng = np.random.default_rng(seed)
    signs = (rng.integers(0, 2, n) * 2 - 1).astype(np.int8)
    cols = np.sort(rng.choice(n, d, replace=False)).astype(np.int32)
    return signs, cols


def test_srht_columns_orthonormal_and_entries():
    n, d = 256, 40
    signs, cols = _draw(n, d, 3)
    om = srht.srht_dense(signs, cols)
    np.testing.assert_allclose(om.T @ om, np.eye(d), atol=1e-14)
    ref = signs[:, None].astype(np.float64) * hadamard(n)[:, cols] / np.sqrt(n)
    np.testing.assert_array_equal(om, ref)
    rows = np.array([0, 5, 255, 128, 77])
    np.testing.assert_array_equal(srht.entries(signs, cols, rows), ref[rows])


def test_right_and_left_apply_match_dense():
    n, d = 512, 33
    signs, cols = _draw(n, d, 4)
    rng = np.random.default_rng(5)
    m = rng.standard_normal((7, n))
    q = rng.standard_normal((n, 5))
    om = signs[:, None].astype(np.float64) * hadamard(n)[:, cols] / np.sqrt(n)
    np.testing.assert_allclose(srht.right_apply(m, signs, cols), m @ om, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(srht.left_apply_t(q, signs, cols), om.T @ q, rtol=1e-12, atol=1e-12)
