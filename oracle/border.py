"""FP64 reference for the protective border (Sec. 2.3).  TEST INFRASTRUCTURE ONLY.

The border added around the target source region is sized from the
probability density of the stars' deflection perturbation phi (the deflection
of N point masses minus its mean, in units of phi_0 = sqrt(kappa_*)).  The
paper compares its numerical densities with the closed form of Katz, Balbus
and Paczynski (1986) (their Eq. 13; the paper's Eq. 10) for the density of
the vector phi:

    rho_N(phi) = 1/(2 pi phi_0^2) int_0^inf x dx J_0(x phi/phi_0)
                 exp[-(x^2/2) ln(c N^(1/2) / x)],          c = 3.05,

and with the same form at c = 1.454 (the paper's Eq. 11, the modified
characteristic function exp[-(N k^2/2) ln(1.454/k)], which is the above with
x = k N^(1/2)).

Reading of the paper: the exponent
f(x) = -(x^2/2) ln(c sqrt(N)/x) falls to its minimum -c^2 N/(4e) at
x_m = c sqrt(N) e^(-1/2) and grows again beyond (the approximation behind it
holds for x << c sqrt(N)); the integral is taken over [0, x_m], which leaves
out less than exp(-c^2 N/(4e)) (< 4e-9 for N >= 100 at either c).

Functions:
  char_fn(x, n, c)          exp f(x), the characteristic function at |k| = x
  radial_pdf(u, n, c)       p(u) = 2 pi u rho(u phi_0) phi_0^2: density of
                            u = |phi|/phi_0 (integrates to 1 over u >= 0)
  radial_cdf(u, n, c)       P(|phi|/phi_0 <= u)

Pinned by tests/test_oracle_border.py: normalisation; the point-mass tail
p(u) ~ 2/u^3 (a star closer than 1/(u phi_0) gives |phi| > u phi_0, and
there are kappa_*/pi stars per unit area: P(> u) -> 1/u^2); the inverse
Hankel transform of p returning exp f; the CDF as the integral of p.
"""
import math

import numpy as np
from scipy import integrate, special

KATZ_C = 3.05        # Katz, Balbus & Paczynski (1986), Eq. 13
MODIFIED_C = 1.454   # the paper's Eq. 11


def x_max(n, c):
    """Upper limit of the x integral: where the exponent is smallest."""
    return c * math.sqrt(n) * math.exp(-0.5)


def char_fn(x, n, c):
    """exp[-(x^2/2) ln(c sqrt(n)/x)] for 0 <= x <= x_max (1 at x = 0)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    pos = x > 0
    xp = x[pos]
    out[pos] = np.exp(-0.5 * xp * xp * np.log(c * math.sqrt(n) / xp))
    return out


def _integrand_pdf(x, u, n, c):
    return x * special.j0(x * u) * char_fn(np.array([x]), n, c)[0]


def radial_pdf(u, n, c):
    """Density of u = |phi|/phi_0: p(u) = u int_0^{x_m} x J0(x u) exp f(x) dx.

    (rho(phi) phi_0^2 = (1/2pi) int x J0 exp f dx; p(u) = 2 pi u rho phi_0^2.)"""
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    xm = x_max(n, c)
    out = np.empty_like(u)
    for k, uk in enumerate(u):
        # J0 oscillates with period ~2 pi/u: split the range accordingly
        pieces = max(8, int(xm * max(uk, 1e-3) / math.pi) + 1)
        edges = np.linspace(0.0, xm, min(pieces, 4000) + 1)
        s = 0.0
        for a, b in zip(edges[:-1], edges[1:]):
            s += integrate.quad(_integrand_pdf, a, b, args=(uk, n, c), limit=200,
                                epsabs=1e-13, epsrel=1e-10)[0]
        out[k] = uk * s
    return out


def _integrand_cdf(x, u, n, c):
    # int_0^u p(v) dv = u int x^0 J1(x u) exp f(x) dx  (since d/du[u J1(xu)] = x u J0(xu))
    return special.j1(x * u) * char_fn(np.array([x]), n, c)[0]


def radial_cdf(u, n, c):
    """P(|phi|/phi_0 <= u) = u int_0^{x_m} J1(x u) exp f(x) dx."""
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    xm = x_max(n, c)
    out = np.empty_like(u)
    for k, uk in enumerate(u):
        pieces = max(8, int(xm * max(uk, 1e-3) / math.pi) + 1)
        edges = np.linspace(0.0, xm, min(pieces, 4000) + 1)
        s = 0.0
        for a, b in zip(edges[:-1], edges[1:]):
            s += integrate.quad(_integrand_cdf, a, b, args=(uk, n, c), limit=200,
                                epsabs=1e-13, epsrel=1e-10)[0]
        out[k] = uk * s
    return out
