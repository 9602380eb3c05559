"""Lens sets: positions uniform in a rectangle the caller supplies, masses equal
or drawn from a power-law (Salpeter-type) mass function.

The paper's flow chart generates "random positions and mass for lenses
following certain mass distributions" with mass-function parameters
(M_min, M_max, alpha) (Sec. 2.4, Input parameters / Generate lenses).  Angles
are in units of the Einstein angle of the MEAN mass (Eq. 3), so masses are
returned divided by the mass function's mean: m_i = M_i / <M>.
"""
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .rng import uniform01

SALPETER_SLOPE = 2.35   # dN/dM ~ M^-2.35 (Salpeter 1955); the paper gives no number


@dataclass
class Lenses:
    x: np.ndarray                 # float64, theta_1 of each lens
    y: np.ndarray                 # float64, theta_2 of each lens
    m: Optional[np.ndarray]       # float64 masses in units of <M>; None = all 1

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def masses(self) -> np.ndarray:
        return np.ones(self.n) if self.m is None else self.m


def salpeter_mean_mass(m_min: float, m_max: float, slope: float = SALPETER_SLOPE) -> float:
    """Mean of dN/dM ~ M^-slope on [m_min, m_max] (slope != 1, 2)."""
    a, b = 1.0 - slope, 2.0 - slope
    return (a / b) * (m_max ** b - m_min ** b) / (m_max ** a - m_min ** a)


def _salpeter_masses(u: np.ndarray, m_min: float, m_max: float, slope: float) -> np.ndarray:
    a = 1.0 - slope
    lo, hi = m_min ** a, m_max ** a
    return (lo + u * (hi - lo)) ** (1.0 / a)


def uniform_lenses(n: int, rect, seed: int, mass: str = "unit",
                   m_min: float = 0.1, m_max: float = 1.0,
                   slope: float = SALPETER_SLOPE) -> Lenses:
    """n lenses uniform in rect = (a1, a2, b1, b2).

    Streams: 0 -> theta_1, 1 -> theta_2, 2 -> mass.  mass = "unit" gives
    m = None (all ones); mass = "salpeter" draws from the power law on
    [m_min, m_max] by inverting its CDF and divides by the analytic mean.
    """
    a1, a2, b1, b2 = (float(v) for v in rect)
    x = a1 + uniform01(seed, 0, n) * (a2 - a1)
    y = b1 + uniform01(seed, 1, n) * (b2 - b1)
    if mass == "unit":
        m = None
    elif mass == "salpeter":
        m = _salpeter_masses(uniform01(seed, 2, n), m_min, m_max, slope)
        m = m / salpeter_mean_mass(m_min, m_max, slope)
    else:
        raise ValueError(f"unknown mass function {mass!r}")
    return Lenses(np.ascontiguousarray(x), np.ascontiguousarray(y), m)


def disc_lenses(n: int, radius: float, seed: int, mass: str = "unit",
                m_min: float = 0.1, m_max: float = 1.0,
                slope: float = SALPETER_SLOPE) -> Lenses:
    """n lenses uniform in the disc of the given radius about the origin (the
    circular lens plane): r = radius sqrt(u0), angle 2 pi u1; streams 0/1 as
    for the rectangle, stream 2 for masses."""
    r = float(radius) * np.sqrt(uniform01(seed, 0, n))
    a = 2.0 * np.pi * uniform01(seed, 1, n)
    x, y = r * np.cos(a), r * np.sin(a)
    if mass == "unit":
        m = None
    elif mass == "salpeter":
        m = _salpeter_masses(uniform01(seed, 2, n), m_min, m_max, slope)
        m = m / salpeter_mean_mass(m_min, m_max, slope)
    else:
        raise ValueError(f"unknown mass function {mass!r}")
    return Lenses(np.ascontiguousarray(x), np.ascontiguousarray(y), m)
