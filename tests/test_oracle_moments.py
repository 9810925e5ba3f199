"""Pins of the BDIM kernel moments against closed forms and independent quadrature."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import kernel, mu0, mu1
from oracle.moments import kernel_eps


@pytest.mark.parametrize("eps", [1.0, 2.0, 0.5])
def test_moment_end_values(eps):
    assert mu0(-eps, eps) == pytest.approx(0.0, abs=1e-15)
    assert mu0(0.0, eps) == pytest.approx(0.5, abs=1e-15)
    assert mu0(eps, eps) == pytest.approx(1.0, abs=1e-15)
    assert mu0(-3 * eps, eps) == pytest.approx(0.0, abs=1e-16)
    assert mu0(3 * eps, eps) == pytest.approx(1.0, abs=1e-16)
    assert mu1(-eps, eps) == pytest.approx(0.0, abs=1e-15)
    assert mu1(eps, eps) == pytest.approx(0.0, abs=1e-15)
    # mu1(0) = eps (1/4 - 1/pi^2) ~ 0.148679 eps
    assert mu1(0.0, eps) == pytest.approx(eps * (0.25 - 1.0 / math.pi ** 2), rel=1e-14)
    assert mu1(0.0, 1.0) == pytest.approx(0.148679, abs=1e-6)
    # beyond the support the moments are the full integrals, exactly (int K = 1, int s K = 0)
    for d in (eps, 1.5 * eps, 40.0 * eps):
        assert mu0(d, eps) == 1.0 and mu1(d, eps) == 0.0 and mu1(-d, eps) == 0.0
        assert mu0(-d, eps) == 0.0


def test_kernel_unit_integral():
    val, _ = integrate.quad(lambda s: float(kernel(s)), -1.0, 1.0)
    assert val == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("s", np.linspace(-0.97, 0.97, 9))
def test_moments_equal_quadrature(s):
    # mu0 = int_{-1}^{s} K ;  mu1 = -eps int_{-1}^{s} s' K(s') ds'   (independent quadrature)
    eps = 1.5
    m0, _ = integrate.quad(lambda q: float(kernel(q)), -1.0, s, epsabs=1e-14)
    m1, _ = integrate.quad(lambda q: q * float(kernel(q)), -1.0, s, epsabs=1e-14)
    assert mu0(s * eps, eps) == pytest.approx(m0, abs=1e-12)
    assert mu1(s * eps, eps) == pytest.approx(-eps * m1, abs=1e-12)


def test_moment_derivatives():
    # d mu0/dd = K_eps(d);  d mu1/dd = -(d/eps) K(d/eps)  (central differences)
    eps = 1.0
    d = np.linspace(-0.95, 0.95, 23)
    h = 1e-6
    dm0 = (mu0(d + h, eps) - mu0(d - h, eps)) / (2 * h)
    dm1 = (mu1(d + h, eps) - mu1(d - h, eps)) / (2 * h)
    np.testing.assert_allclose(dm0, kernel_eps(d, eps), atol=1e-8)
    np.testing.assert_allclose(dm1, -(d / eps) * kernel(d / eps), atol=1e-8)


def test_mu0_is_smoothed_heaviside():
    # symmetric smoothing: mu0(d) + mu0(-d) = 1, mu1 even
    d = np.linspace(-2, 2, 41)
    np.testing.assert_allclose(mu0(d) + mu0(-d), 1.0, atol=1e-15)
    np.testing.assert_allclose(mu1(d), mu1(-d), atol=1e-15)
