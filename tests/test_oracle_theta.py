"""Pins for the oracle's Matern covariance (Section 4.4 Matern definition)."""
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy.special import gamma, kv
from scipy.spatial import distance_matrix

import oracle as O
from paper_1706_02205_amd import workloads as W


def matern_bessel(r, nu, ell):
    """The general Matern formula with the modified Bessel function K_nu."""
    z = np.sqrt(2 * nu) * r / ell
    return 2 ** (1 - nu) / gamma(nu) * z ** nu * kv(nu, z)


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
@pytest.mark.parametrize("ell", [0.05, 0.2, 1.0])
def test_closed_forms_match_bessel_definition(nu, ell):
    r = np.logspace(-4, 1.3, 400) * ell
    got = O.matern(r, nu, ell)
    ref = matern_bessel(r, nu, ell)
    np.testing.assert_allclose(got, ref, rtol=2e-13, atol=0)
    assert O.matern(np.array([0.0]), nu, ell)[0] == 1.0


def test_exponential_is_correctly_rounded():
    """exp(-a) (nu=1/2, l=1) equals the 60-digit decimal exp rounded to double."""
    getcontext().prec = 60
    a = np.random.Generator(np.random.PCG64(3)).uniform(0.0, 60.0, 20000)
    got = O.matern(a, 0.5, 1.0)
    ref = np.array([float(Decimal(-float(v)).exp()) for v in a])
    assert np.array_equal(got, ref)


def test_unsupported_smoothness_rejected():
    with pytest.raises(ValueError):
        O.matern(np.array([1.0]), 1.0, 0.2)


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_theta_on_pattern(nu):
    x = W.uniform_points(300, 3, 5)
    P = O.pattern(x, 2.0)
    th = O.theta_on_pattern(P, nu, 0.3)
    cols = np.repeat(np.arange(P.n), np.diff(P.colptr))
    D = distance_matrix(P.xh, P.xh)
    ref = matern_bessel(D[P.rowidx, cols], nu, 0.3)
    diag = P.rowidx == cols
    assert np.all(th[diag] == 1.0)
    np.testing.assert_allclose(th[~diag], ref[~diag], rtol=1e-12)
