"""Workload descriptions (inputs only, no derived geometry).

Each workload is what a user of the method types in (Sec. 2.4, Input
parameters): kappa_*, the smooth convergence kappa_c, gamma, the source side
S in Einstein radii, pixels per side, rays per pixel (or a total ray count),
the mass function and a seed.  Source sides quoted with 4-5 digits were chosen
so that the paper's lens-count rule gives the stated N_* (1e5 or 1e6 lenses);
everything else is derived by the side that runs the workload.
"""
from dataclasses import dataclass, replace
from typing import List

import numpy as np

from .rng import uniform01

SEED_BASE = 220410871


@dataclass(frozen=True)
class Workload:
    name: str
    kappa_star: float
    kappa_c: float
    gamma: float
    source_side: float
    npix: int
    rays_per_pixel: float = 0.0      # N_av
    n_rays: int = 0                  # total rays; overrides N_av when > 0
    mass: str = "unit"               # "unit" or "salpeter"
    m_min: float = 0.1
    m_max: float = 1.0
    level2_ray_multiple: float = 0.0  # > 0: level-2 spacing = this many ray spacings
    seed: int = SEED_BASE

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# Plain brute-force map, FP64: 2048^2 rays over the prolate shooting rectangle.
CFG1 = Workload("cfg1_fp64_direct", 0.3, 0.0, 0.3, 10.0, 256,
                n_rays=2048 * 2048, seed=SEED_BASE + 1)

# Direct-sum and grid-interpolated map, 4096^2 pixels, 100 rays per pixel,
# coarse deflection grid at 16 ray spacings.  S = 25 as stated (N_* = 4450 by
# the lens-count rule) ...
CFG2 = Workload("cfg2_s25", 0.45, 0.05, 0.45, 25.0, 4096,
                rays_per_pixel=100.0, level2_ray_multiple=16.0,
                seed=SEED_BASE + 2)
# ... and the same kappa/gamma at N_* = 1e5 (S derived: 168.69).
CFG2T = CFG2.with_(name="cfg2_n1e5", source_side=168.69)

# Large regime: N_* = 1e6 Salpeter [0.1, 1] M_sun, 10000^2 pixels, ~1e11 rays.
CFG3 = Workload("cfg3_n1e6_salpeter", 0.6, 0.0, 0.6, 1007.8, 10000,
                rays_per_pixel=1000.0, mass="salpeter", m_min=0.1, m_max=1.0,
                seed=SEED_BASE + 3)

# Learned far-field workload: kappa_c = 0.05 keeps it off the critical line
# (kappa_* = gamma = 0.5 with kappa_c = 0 has 1 - kappa - gamma = 0).
CFG5 = Workload("cfg5_n1e6_learned", 0.5, 0.05, 0.5, 532.16, 8192,
                rays_per_pixel=100.0, seed=SEED_BASE + 5)
CFG5_LITERAL = CFG5.with_(name="cfg5_literal_critical", kappa_c=0.0)

ALL = {w.name: w for w in (CFG1, CFG2, CFG2T, CFG3, CFG5)}


@dataclass(frozen=True)
class BatchDraw:
    """One map of the batched workload before its source side is derived."""
    index: int
    kappa_star: float
    kappa_c: float
    gamma: float
    n_star_target: int
    npix: int
    rays_per_pixel: float
    seed: int


def batch_draws(n_maps: int = 64, seed: int = SEED_BASE + 4,
                min_lambda: float = 0.05) -> List[BatchDraw]:
    """Draws for the batched workload: kappa_* ~ U[0.1, 0.8], gamma ~ U[0.1, 0.8],
    kappa_c in {0, 0.2}, N_* = 10^U[3, 5], npix in {1024, 2048, 4096},
    100 rays per pixel.  Draws with min |1 - kappa -/+ gamma| < min_lambda are
    rejected (they sit too close to a critical line to size a rectangle)."""
    out: List[BatchDraw] = []
    k = 0
    while len(out) < n_maps:
        u = uniform01(seed, 7, 5, offset=5 * k)
        ks = 0.1 + 0.7 * u[0]
        g = 0.1 + 0.7 * u[1]
        kc = 0.0 if u[2] < 0.5 else 0.2
        nstar = int(round(10.0 ** (3.0 + 2.0 * u[3])))
        npix = (1024, 2048, 4096)[min(2, int(3 * u[4]))]
        kap = ks + kc
        if min(abs(1 - kap - g), abs(1 - kap + g)) >= min_lambda:
            out.append(BatchDraw(len(out), float(ks), kc, float(g), nstar, npix,
                                 100.0, (SEED_BASE + 4) * 1000 + len(out)))
        k += 1
    return out
