"""Oracle geometry: the sizing rules of the paper's flow chart (Sec. 2.4), in
plain FP64 Python.  Test infrastructure only.

Rules (each line cites the step it follows):
  kappa = kappa_s + kappa_*                                   (Eq. 2)
  P = 10 sqrt(kappa_*)                  "Calculate the size of the Protective Border"
  I_x = (S + 2P)/|1 - kappa - gamma|,  I_y = (S + 2P)/|1 - kappa + gamma|   (same step)
  N_rays = N_av N_pix;  dx3 = sqrt(I_x I_y / N_rays)          (level-3 resolution)
  L0 = sqrt(I_x I_y / N_*);  dx1 = min(L0, min(I_x, I_y)/10)  (level-1 resolution)
  dx2 = dx1 / 20                                               (level-2 resolution)
  Mag_ij = N_ij S_I / S_S                                      (magnification step)

Readings where the paper is silent:
  - the rectangle is centred at the origin;
  - the ray grid has nx = round(I_x/dx3), ny = round(I_y/dx3) columns/rows,
    rays at cell centres, so S_I = (I_x/nx)(I_y/ny);
  - the level-1 grid tiles the rectangle exactly with n1x = ceil(I_x/dx1)
    by n1y = ceil(I_y/dx1) cells (cells of side <= dx1); each cell is split into
    q x q level-2 subcells, q = round(dx1/dx2), level-2 points at subcell centres;
  - the source map is [-S/2, S/2)^2 with S/npix pixels.
"""
import math
from dataclasses import dataclass


class CriticalLineError(ValueError):
    """|1 - kappa -/+ gamma| is ~0: the shooting rectangle is unbounded."""


def _round_half_up(v: float) -> int:
    return int(math.floor(v + 0.5))


@dataclass(frozen=True)
class Geometry:
    kappa_star: float
    kappa_c: float
    gamma: float
    kappa: float
    source_side: float
    npix: int
    border: float
    ix: float
    iy: float
    a1: float
    a2: float
    b1: float
    b2: float
    n_rays_target: int
    dx3: float
    nx: int
    ny: int
    n_lens: int
    dx1: float
    n1x: int
    n1y: int
    dx2: float
    q: int
    dpix: float
    s_img: float
    s_src: float
    mu_th: float
    sheet: bool

    @property
    def n_rays(self) -> int:
        return self.nx * self.ny

    @property
    def ray_dx(self) -> float:
        return (self.a2 - self.a1) / self.nx

    @property
    def ray_dy(self) -> float:
        return (self.b2 - self.b1) / self.ny

    @property
    def rect(self):
        return (self.a1, self.a2, self.b1, self.b2)

    @property
    def lens_radius(self) -> float:
        """Circular lens plane: radius of the image rectangle's circumscribed
        circle (Sec. 2.2); 0 for the rectangle."""
        return 0.5 * math.hypot(self.ix, self.iy) if self.circle else 0.0

    @property
    def n_stars_expected(self) -> int:
        """Lens count that fills the lens plane at density kappa_* with unit mean
        mass: the sheet of Appendix A has A = kappa_*/pi per unit area, i.e.
        kappa_* I_x I_y / pi Einstein masses (kappa_* R^2 for the circle)."""
        if self.circle:
            return _round_half_up(self.kappa_star * self.lens_radius ** 2)
        return _round_half_up(self.kappa_star * self.ix * self.iy / math.pi)

    l2_spacing_arg: float = 0.0        # explicit level-2 spacing, 0 = rule
    l2_ray_multiple_arg: float = 0.0   # level-2 spacing in ray spacings, 0 = rule
    circle: bool = False               # circular lens plane, sheet -kappa_* theta (Eq. 9)

    def with_lens_count(self, n_lens: int) -> "Geometry":
        """Same inputs, geometry re-derived for n_lens lenses (dx1 depends on N_*)."""
        return geometry(self.kappa_star, self.kappa_c, self.gamma, self.source_side,
                        self.npix, n_rays=self.n_rays_target, border=self.border,
                        n_lens=n_lens, level2_spacing=self.l2_spacing_arg,
                        level2_ray_multiple=self.l2_ray_multiple_arg, sheet=self.sheet,
                        circle=self.circle)


def geometry(kappa_star, kappa_c, gamma, source_side, npix, rays_per_pixel=None,
             n_rays=None, border=None, n_lens=0, level2_spacing=None,
             level2_ray_multiple=None, crit_eps=1e-3, sheet=True, circle=False) -> Geometry:
    kappa = kappa_star + kappa_c
    lam1 = 1.0 - kappa - gamma
    lam2 = 1.0 - kappa + gamma
    if abs(lam1) < crit_eps or abs(lam2) < crit_eps:
        raise CriticalLineError(f"|1-kappa-gamma|={abs(lam1):.3g}, |1-kappa+gamma|={abs(lam2):.3g}")
    P = 10.0 * math.sqrt(kappa_star) if border is None or border < 0 else float(border)
    S = float(source_side)
    ix = (S + 2.0 * P) / abs(lam1)
    iy = (S + 2.0 * P) / abs(lam2)
    if n_rays is None or n_rays <= 0:
        n_rays = _round_half_up(rays_per_pixel * npix * npix)
    dx3 = math.sqrt(ix * iy / n_rays)
    nx = max(1, _round_half_up(ix / dx3))
    ny = max(1, _round_half_up(iy / dx3))
    short = min(ix, iy) / 10.0
    dx1 = short if n_lens <= 0 else min(math.sqrt(ix * iy / n_lens), short)
    n1x = max(1, math.ceil(ix / dx1 - 1e-9))
    n1y = max(1, math.ceil(iy / dx1 - 1e-9))
    if level2_spacing is not None and level2_spacing > 0:
        dx2 = float(level2_spacing)
    elif level2_ray_multiple is not None and level2_ray_multiple > 0:
        dx2 = level2_ray_multiple * dx3
    else:
        dx2 = dx1 / 20.0
    q = max(1, _round_half_up(dx1 / dx2))
    dpix = S / npix
    s_img = (ix / nx) * (iy / ny)
    g = Geometry(kappa_star=kappa_star, kappa_c=kappa_c, gamma=gamma, kappa=kappa,
                 source_side=S, npix=int(npix), border=P, ix=ix, iy=iy,
                 a1=-0.5 * ix, a2=0.5 * ix, b1=-0.5 * iy, b2=0.5 * iy,
                 n_rays_target=int(n_rays), dx3=dx3, nx=nx, ny=ny, n_lens=int(n_lens),
                 dx1=dx1, n1x=n1x, n1y=n1y, dx2=dx2, q=q, dpix=dpix, s_img=s_img,
                 s_src=dpix * dpix, mu_th=1.0 / (lam1 * lam2), sheet=bool(sheet),
                 l2_spacing_arg=float(level2_spacing or 0.0),
                 l2_ray_multiple_arg=float(level2_ray_multiple or 0.0), circle=bool(circle))
    return g


def source_side_for_lens_count(kappa_star, kappa_c, gamma, n_star, border=None) -> float:
    """Inverse of the lens-count rule: the source side S whose rectangle holds
    n_star unit-mean-mass lenses at density kappa_* (N_* = kappa_* I_x I_y / pi)."""
    kappa = kappa_star + kappa_c
    lam = abs((1.0 - kappa - gamma) * (1.0 - kappa + gamma))
    P = 10.0 * math.sqrt(kappa_star) if border is None or border < 0 else float(border)
    return math.sqrt(n_star * math.pi * lam / kappa_star) - 2.0 * P
