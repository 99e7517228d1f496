"""Pins of the oracle's softening kernel against its definition.

The kernel is the M4 cubic spline with compact support h (a reading: the
paper only says that softening follows the hydro kernel length, Sec. 3).
The oracle's force factor f and its derivative D are algebraic rewrites; here
they are checked against quantities computed from the density kernel W alone:
the enclosed mass by numerical quadrature, and D = f'/r by finite differences.
"""
import numpy as np
import pytest
from scipy import integrate


def w_m4(u):
    """Dimensionless M4 kernel shape, written from its textbook definition."""
    u = np.asarray(u, dtype=float)
    return np.where(u < 0.5, 1 - 6 * u**2 + 6 * u**3, np.where(u < 1, 2 * (1 - u) ** 3, 0.0))


def W_m4(r, h):
    return 8.0 / (np.pi * h**3) * w_m4(r / h)


def enclosed_mass(r, h):
    val, _ = integrate.quad(lambda s: 4 * np.pi * s * s * W_m4(s, h), 0.0, min(r, h),
                            points=[0.5 * h] if r > 0.5 * h else None, epsabs=0.0,
                            epsrel=1e-13, limit=200)
    return val


def test_kernel_normalised(orc):
    assert enclosed_mass(1.0, 1.0) == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("h", [1.0, 0.01, 3.7e-3])
def test_force_factor_is_enclosed_mass_over_r3(orc, h):
    r = h * np.array([1e-3, 0.1, 0.3, 0.49, 0.5, 0.51, 0.7, 0.9, 0.999, 1.0, 1.5, 4.0])
    f, D, W = orc.kernel(r, h)
    mu = np.array([enclosed_mass(ri, h) for ri in r])
    np.testing.assert_allclose(f * r**3, mu, rtol=2e-12, atol=1e-14)
    np.testing.assert_allclose(W, W_m4(r, h), rtol=1e-13, atol=0)


def test_enclosed_mass_at_half_and_one(orc):
    # mu(1/2) = 19/30, mu(1) = 1: the piecewise forms join continuously
    h = 1.0
    f, _, _ = orc.kernel(np.array([0.5 - 1e-12, 0.5 + 1e-12, 1 - 1e-12, 1 + 1e-12]), h)
    r = np.array([0.5, 0.5, 1.0, 1.0])
    np.testing.assert_allclose(f * r**3, [19 / 30, 19 / 30, 1, 1], rtol=1e-10)


@pytest.mark.parametrize("h", [1.0, 0.05])
def test_D_is_fprime_over_r(orc, h):
    r = h * np.array([0.05, 0.2, 0.45, 0.55, 0.8, 0.95, 1.2, 3.0])
    d = 1e-6 * h
    fp, _, _ = orc.kernel(r + d, h)
    fm, _, _ = orc.kernel(r - d, h)
    _, D, _ = orc.kernel(r, h)
    fd = (fp - fm) / (2 * d) / r
    np.testing.assert_allclose(D, fd, rtol=1e-7)


def test_newtonian_outside_support(orc):
    h = 0.01
    r = np.array([0.01, 0.02, 0.5, 3.0])
    f, D, W = orc.kernel(r, h)
    np.testing.assert_allclose(f, r**-3, rtol=1e-14)
    np.testing.assert_allclose(D, -3 * r**-5, rtol=1e-14)
    assert np.all(W == 0)


def test_finite_at_zero_separation(orc):
    h = 0.1
    f, D, W = orc.kernel(np.array([0.0]), h)
    assert f[0] == pytest.approx(32.0 / 3.0 / h**3, rel=1e-14)
    assert D[0] == pytest.approx(-384.0 / 5.0 / h**5, rel=1e-14)
    assert W[0] == pytest.approx(8 / np.pi / h**3, rel=1e-14)


def test_poisson_kernel_identity(orc):
    # 3 f + r f' = 3 f + D r^2 = 4 pi W  (the trace of the pair tidal tensor)
    h = 0.2
    r = np.linspace(0.0, 1.5 * h, 301)
    f, D, W = orc.kernel(r, h)
    np.testing.assert_allclose(3 * f + D * r**2, 4 * np.pi * W_m4(r, h), rtol=1e-11, atol=1e-9)
