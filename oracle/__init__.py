"""FP64 CPU oracle for the inverse-ray-shooting path of arXiv 2204.10871.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP library (paper_2204_10871_amd) and does not import it.

  geometry.py  -- the printed sizing rules (protective border, rectangle, ray
                  grid, level-1/2/3 resolutions, pixel areas).
  irs_oracle.c -- O-1 (direct definition of Eq. 6 + Appendix A + binning) and
                  O-2 (the three-level-grid interpolation, step by step).
  border.py    -- the deflection-perturbation density behind the protective
                  border (Sec. 2.3, Eqs. 10-11), by direct integration.
  learned.py   -- FP64 reference of the learned far-field interpolant (network,
                  base interpolant, local data); orc_far_point gives its exact
                  samples.

Parity status of each function is listed in its docstring ("pinned by ...").
"""
from .geometry import Geometry, geometry, CriticalLineError, source_side_for_lens_count
from .core import (build, load, sheet_I, alpha_points, shoot_direct, level1,
                   level2, level2_grid, shoot_interp, shoot_interp_rays, sheet_taylor, setup_of, far_point)

__all__ = ["Geometry", "geometry", "CriticalLineError", "source_side_for_lens_count",
           "build", "load", "sheet_I", "alpha_points", "shoot_direct", "level1",
           "level2", "level2_grid", "shoot_interp", "shoot_interp_rays", "sheet_taylor", "setup_of", "far_point"]
