// Host-side plan geometry (no HIP dependency).
//
// Sizing rules follow the flow chart of Sec. 2.4: protective border
// P = 10 sqrt(kappa_*), rectangle I_x = (S+2P)/|1-kappa-gamma|,
// I_y = (S+2P)/|1-kappa+gamma|; level-1 resolution min(L0, min(I_x,I_y)/10)
// with L0 = sqrt(I_x I_y / N_*); level-2 resolution dx1/20; level-3 (ray)
// resolution sqrt(I_x I_y / N_rays) with N_rays = N_av N_pix.
#pragma once

#include <cstdint>
#include <string>

#include "../../include/irs.h"

namespace irs {

struct HostGeometry {
    irs_geometry_info info;
    double kappa_star, kappa_c, gamma, source_side;
    int64_t npix;
    bool sheet;
    bool circle;                  // IRS_CIRCLE: circular lens plane, sheet -kappa_* theta
};

// Fills `out` or returns an error status with a message in `err`.
irs_status derive_geometry(const irs_params &p, int64_t n_lens, HostGeometry &out,
                           std::string &err);

// Ray rows (axis 1) or ray columns (axis 0) [first, last) whose level-2
// points lie in level-1 row or column c.  Ray row j lies in level-2 row
// floor((2j+1) n1y q / (2 ny)), a non-decreasing function of j.
void level1_span(const irs_geometry_info &g, int axis, int64_t c, int64_t &first, int64_t &last);

// Source side S whose rectangle holds n_star lenses by the lens-count rule
// (the smallest S, to bisection precision, with n_stars_expected >= n_star;
// every other field of p is used as given).
irs_status source_side_for_lens_count(const irs_params &p, int64_t n_star, double &side,
                                      std::string &err);

}  // namespace irs
