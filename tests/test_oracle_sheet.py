"""Pins of the oracle's rectangle sheet (Appendix A) against mathematics that
does not go through its closed forms: 2-D quadrature of the defining integral,
Gauss's law (divergence), irrotationality, symmetry, the infinite-slab limit,
and the analytic structure used by the level-2 Taylor coefficients."""
import math

import numpy as np
import pytest
from scipy import integrate


RECT = (-3.7, 5.1, -1.3, 2.2)   # deliberately off-centre and non-square


def _quad_I(rect, x, y):
    """Appendix A's defining integrals (A = 1) by adaptive quadrature, split at
    the evaluation point so each piece has its integrable singularity at a corner."""
    a1, a2, b1, b2 = rect
    xs = [a1, x, a2] if a1 < x < a2 else [a1, a2]
    ys = [b1, y, b2] if b1 < y < b2 else [b1, b2]
    f1 = lambda yp, xp: (x - xp) / ((x - xp) ** 2 + (y - yp) ** 2)
    f2 = lambda yp, xp: (y - yp) / ((x - xp) ** 2 + (y - yp) ** 2)
    I1 = I2 = 0.0
    for i in range(len(xs) - 1):
        for j in range(len(ys) - 1):
            I1 += integrate.dblquad(f1, xs[i], xs[i + 1], ys[j], ys[j + 1],
                                    epsabs=1e-11, epsrel=1e-11)[0]
            I2 += integrate.dblquad(f2, xs[i], xs[i + 1], ys[j], ys[j + 1],
                                    epsabs=1e-11, epsrel=1e-11)[0]
    return I1, I2


@pytest.mark.parametrize("pt", [(0.3, 0.4), (-3.5, -1.1), (4.9, 2.0), (1.0, -1.29),
                                (7.0, 4.0), (-5.0, 0.5)])
def test_closed_form_matches_quadrature(orc, pt):
    """Inside (incl. near corners) and outside the rectangle."""
    I1, I2 = orc.sheet_I(RECT, [pt[0]], [pt[1]])
    q1, q2 = _quad_I(RECT, *pt)
    assert abs(I1[0] - q1) < 2e-8 * max(1.0, abs(q1))
    assert abs(I2[0] - q2) < 2e-8 * max(1.0, abs(q2))


def _grad(orc, rect, x, y, h=1e-4):
    Ix1, Iy1 = orc.sheet_I(rect, [x + h, x - h, x, x], [y, y, y + h, y - h])
    dI1dx = (Ix1[0] - Ix1[1]) / (2 * h)
    dI1dy = (Ix1[2] - Ix1[3]) / (2 * h)
    dI2dx = (Iy1[0] - Iy1[1]) / (2 * h)
    dI2dy = (Iy1[2] - Iy1[3]) / (2 * h)
    return dI1dx, dI1dy, dI2dx, dI2dy


@pytest.mark.parametrize("pt", [(0.1, 0.2), (-3.0, -1.0), (4.5, 1.9), (2.0, 0.0)])
def test_divergence_and_curl_inside(orc, pt):
    """A positive unit-density sheet has div = 2 pi (Poisson, A = 1) and no curl;
    the oracle's deflection -(kappa_*/pi)(I1, I2) therefore has div = -2 kappa_*."""
    d11, d12, d21, d22 = _grad(orc, RECT, *pt)
    assert abs((d11 + d22) - 2 * math.pi) < 1e-6
    assert abs(d12 - d21) < 1e-6


def test_divergence_outside_is_zero(orc):
    d11, d12, d21, d22 = _grad(orc, RECT, 8.0, 5.0)
    assert abs(d11 + d22) < 1e-7 and abs(d12 - d21) < 1e-7


def test_square_centre_no_shear(orc):
    """At the centre of a square the field is isotropic: I = pi theta to first order."""
    sq = (-2.0, 2.0, -2.0, 2.0)
    I1, I2 = orc.sheet_I(sq, [0.0], [0.0])
    assert abs(I1[0]) < 1e-14 and abs(I2[0]) < 1e-14
    d11, d12, d21, d22 = _grad(orc, sq, 0.0, 0.0)
    assert abs(d11 - math.pi) < 1e-7 and abs(d22 - math.pi) < 1e-7 and abs(d12) < 1e-7


def test_long_strip_is_a_slab(orc):
    """A rectangle much longer in x than in y acts, near its centre, like an
    infinite slab: deflection 2 pi y along y only (A = 1)."""
    strip = (-1e5, 1e5, -1.0, 1.0)
    I1, I2 = orc.sheet_I(strip, [0.0, 0.0], [0.3, -0.7])
    assert np.allclose(I2, [2 * math.pi * 0.3, -2 * math.pi * 0.7], atol=1e-4)
    assert np.all(np.abs(I1) < 1e-4)


def test_circular_limit_of_large_square(orc):
    """Deep inside a large square, near its centre, the sheet approaches the
    circular plane's uniform deflection (Eq. 9 for the negative sheet):
    I ~ pi theta, i.e. alpha_{-kappa} = -kappa theta."""
    sq = (-500.0, 500.0, -500.0, 500.0)
    x = np.array([1.0, -2.0, 3.0])
    y = np.array([0.5, 1.5, -2.5])
    I1, I2 = orc.sheet_I(sq, x, y)
    assert np.allclose(I1, math.pi * x, rtol=1e-5)
    assert np.allclose(I2, math.pi * y, rtol=1e-5)


def _F(orc, g, z):
    I1, I2 = orc.sheet_I(g.rect, [z.real], [z.imag])
    return (I1[0] - 1j * I2[0]) / math.pi


def _small_geometry(orc):
    g = orc.geometry(0.4, 0.1, 0.2, 6.0, 64, n_rays=200 * 200)
    return g.with_lens_count(20)


@pytest.mark.parametrize("corner_off", [2.0 + 1.5j, 1.0 + 3.0j, 4.0 + 0.8j])
def test_sheet_series_is_fifth_order(orc, corner_off):
    """F(z0+h) - [g0 + conj(h) + sum_{k=1..4} g_k h^k] = O(|h|^5): halving h
    divides the remainder by ~32.  A wrong g_k (k <= 4) leaves an O(h^k) term.
    z0 sits at `corner_off` from each of the four corners in turn, and |h| is a
    fraction of the distance to the nearest edge (so z0 + h stays inside, where
    F = conj(z) + G(z)) and large enough that the 5th-order term dominates rounding."""
    g = _small_geometry(orc)
    d = min(corner_off.real, corner_off.imag)
    for sx, sy, cx, cy in ((1, 1, g.a1, g.b1), (-1, 1, g.a2, g.b1),
                           (-1, -1, g.a2, g.b2), (1, -1, g.a1, g.b2)):
        z0 = complex(cx + sx * corner_off.real, cy + sy * corner_off.imag)
        coef = orc.sheet_taylor(g, z0)
        assert abs(coef[0] - _F(orc, g, z0)) < 1e-13
        rem = []
        for f in (0.8, 0.4, 0.2):
            h = f * d * np.exp(0.7j)
            series = coef[0] + np.conj(h) + sum(coef[k] * h ** k for k in range(1, 5))
            rem.append(abs(_F(orc, g, z0 + h) - series))
        assert rem[0] > 1e-9, rem
        assert 22 < rem[0] / rem[1] < 45 and 22 < rem[1] / rem[2] < 45, rem


def test_sheet_first_derivative_by_differences(orc):
    """g_1 = dF/dz = (dF/dx - i dF/dy)/2 from finite differences of the closed form."""
    g = _small_geometry(orc)
    z0 = 0.7 - 0.4j
    h = 1e-5
    dFdx = (_F(orc, g, z0 + h) - _F(orc, g, z0 - h)) / (2 * h)
    dFdy = (_F(orc, g, z0 + 1j * h) - _F(orc, g, z0 - 1j * h)) / (2 * h)
    dz = 0.5 * (dFdx - 1j * dFdy)
    dzbar = 0.5 * (dFdx + 1j * dFdy)
    coef = orc.sheet_taylor(g, z0)
    assert abs(dzbar - 1.0) < 1e-8          # F = conj(z) + G(z) inside
    assert abs(dz - coef[1]) < 1e-8
