"""Pins of the perturbation-density reference (Sec. 2.3, Eqs. 10-11 forms):
properties the closed form must have whatever its implementation."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import border as ob


@pytest.mark.parametrize("n", [100, 10000])
@pytest.mark.parametrize("c", [ob.KATZ_C, ob.MODIFIED_C])
def test_density_integrates_to_one(n, c):
    # char_fn(0) = 1 is the total probability; check it on the density itself
    body = integrate.quad(lambda u: ob.radial_pdf(u, n, c)[0], 0.0, 30.0, limit=400)[0]
    tail = 1.0 / 30.0 ** 2               # P(u > 30) of the point-mass tail
    assert abs(body + tail - 1.0) < 2e-3


@pytest.mark.parametrize("c", [ob.KATZ_C, ob.MODIFIED_C])
def test_point_mass_tail(c):
    # a star closer than 1/(u phi_0) deflects by more than u phi_0; with
    # kappa_*/pi stars per unit area P(> u) -> 1/u^2, so p(u) u^3 -> 2
    # (the approach is O(1/u^2): 2.08 at u = 40, 2.02 at 80)
    u = np.array([80.0, 160.0])
    t = ob.radial_pdf(u, 10000, c) * u ** 3
    assert abs(t[0] - 2.0) < 0.04 and abs(t[1] - 2.0) < 0.012, t
    assert abs(ob.radial_cdf(np.array([80.0]), 10000, c)[0] - (1.0 - 1.0 / 80.0 ** 2)) < 2e-5


@pytest.mark.parametrize("c", [ob.KATZ_C, ob.MODIFIED_C])
def test_cdf_is_the_integral_of_the_density(c):
    for uk in (0.7, 2.5, 6.0):
        direct = integrate.quad(lambda v: ob.radial_pdf(v, 1000, c)[0], 0.0, uk, limit=200)[0]
        assert abs(ob.radial_cdf(np.array([uk]), 1000, c)[0] - direct) < 1e-6


def test_inverse_transform_returns_the_characteristic_function():
    # the 2-d Fourier transform of the density at |k| = x is exp f(x):
    # int_0^inf p(u) J0(x u) du = exp f(x)
    n, c = 1000, ob.MODIFIED_C
    for x in (0.3, 1.0, 2.0):
        val = integrate.quad(lambda u: ob.radial_pdf(u, n, c)[0] * special.j0(x * u), 0.0, 60.0,
                             limit=800)[0]
        assert abs(val - ob.char_fn(np.array([x]), n, c)[0]) < 2e-3


def test_larger_constant_widens_the_core_and_more_stars_too():
    # the log factor is the core's variance: a larger c or N spreads phi
    m = {}
    for n in (100, 10000):
        for c in (ob.MODIFIED_C, ob.KATZ_C):
            F = ob.radial_cdf(np.array([1.0, 2.0]), n, c)
            m[(n, c)] = F
    assert np.all(m[(100, ob.KATZ_C)] < m[(100, ob.MODIFIED_C)])
    assert np.all(m[(10000, ob.MODIFIED_C)] < m[(100, ob.MODIFIED_C)])


def test_gaussian_limit_of_the_core():
    # for the exponent -(x^2/2) L with a constant L the density of u is the
    # Rayleigh law u/L exp(-u^2/(2L)); the closed form with the log frozen at
    # its value near the core's x ~ 1/sqrt(L) must be close to it there
    n, c = 10 ** 8, ob.MODIFIED_C
    L = math.log(c * math.sqrt(n))
    L_eff = L + 0.5 * math.log(L)          # ln(c sqrt(N) / x) at x = 1/sqrt(L)
    u = np.array([2.0, 4.0, 6.0])
    rayleigh = u / L_eff * np.exp(-u * u / (2 * L_eff))
    p = ob.radial_pdf(u, n, c)
    assert np.all(np.abs(p - rayleigh) / rayleigh < 0.15), (p, rayleigh)
