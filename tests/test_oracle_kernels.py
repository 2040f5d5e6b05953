"""Pins of the oracle's covariance kernels (Sec. 5.1, Tables 1-2)."""
import math

import numpy as np
import pytest
from scipy import special
from scipy.spatial.distance import cdist

from oracle import kernels

GRID = np.linspace(0.0, 1.0, 100)[:, None]


def _cond(k, m):
    ev = np.sort(np.linalg.eigvalsh(k))[::-1]
    return ev[0] / ev[m - 1]


def _check(value, kind, printed):
    if kind == "exact":
        assert value == pytest.approx(float(printed), rel=5e-4)
    else:
        assert math.floor(math.log10(value)) == int(printed)


def test_table1_squared_exponential(golden):
    r2 = kernels.sq_dists(GRID, GRID)
    for m, theta2, kind, printed in golden("table1_se_condition.txt"):
        theta2 = float(theta2)
        # theta1 exp(-theta2 r^2) with theta1 = 1 is s = 1, ell = 1/sqrt(2 theta2).
        k = kernels.se(r2, 1.0 / math.sqrt(2.0 * theta2), 1.0)
        _check(_cond(k, int(m)), kind, printed)


def test_table2_matern(golden):
    r = np.sqrt(kernels.sq_dists(GRID, GRID))
    for m, nu, kind, printed in golden("table2_matern_condition.txt"):
        k = kernels.matern_general(r, float(nu), 1.0, 1.0, scale="2sqrtnu")
        _check(_cond(k, int(m)), kind, printed)


def test_table2_printed_scale_is_off():
    # With the printed sqrt(2 nu) argument the nu = 0.5, m = 5 entry is not 38.18.
    r = np.sqrt(kernels.sq_dists(GRID, GRID))
    k = kernels.matern_general(r, 0.5, 1.0, 1.0, scale="sqrt2nu")
    assert abs(_cond(k, 5) - 38.18) > 1.0


def test_matern32_closed_form_matches_bessel():
    rng = np.random.default_rng(0)
    r = np.concatenate([[0.0, 1e-9], rng.uniform(0, 3, 500)])
    ell, s = 0.37, 1.3
    closed = kernels.matern32(r * r, ell, s)
    # Bessel form with nu = 3/2, theta2 = ell, theta1 = s^2, argument sqrt(2 nu) r / ell.
    z = math.sqrt(3.0) * r / ell
    bessel = np.where(z > 0, s * s / (special.gamma(1.5) * 2.0 ** 0.5)
                      * np.where(z > 0, z, 1.0) ** 1.5 * special.kv(1.5, np.where(z > 0, z, 1.0)), s * s)
    np.testing.assert_allclose(closed, bessel, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(kernels.matern_general(r, 1.5, s * s, ell), closed, rtol=1e-13, atol=1e-15)


def test_sq_dists_difference_form_symmetric_nonnegative():
    rng = np.random.default_rng(1)
    x = rng.random((300, 3)).astype(np.float32)
    x[7] = x[3]
    r2 = kernels.sq_dists(x, x)
    assert np.array_equal(r2, r2.T)
    assert (r2 >= 0).all() and r2[7, 3] == 0.0
    np.testing.assert_allclose(r2, cdist(x.astype(np.float64), x.astype(np.float64), "sqeuclidean"),
                               rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("kind", ["se", "matern32"])
def test_kernel_diag_and_dlogell(kind):
    rng = np.random.default_rng(2)
    x = rng.random((50, 2))
    ell, s = 0.3, 1.7
    k = kernels.kernel_matrix(kind, x, x, ell, s)
    np.testing.assert_allclose(np.diag(k), s * s, rtol=1e-15)
    h = 1e-4
    kp = kernels.kernel_matrix(kind, x, x, ell * math.exp(h), s)
    km = kernels.kernel_matrix(kind, x, x, ell * math.exp(-h), s)
    fd = (kp - km) / (2 * h)
    np.testing.assert_allclose(kernels.kernel_matrix_dlogell(kind, x, x, ell, s), fd, rtol=1e-6, atol=1e-9)
