// Host-side plan geometry; see geometry.hpp for the rules it follows.
#include "geometry.hpp"

#include <cmath>
#include <cstdio>

namespace irs {

namespace {

int64_t round_half_up(double v) { return (int64_t)std::floor(v + 0.5); }

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

}  // namespace

irs_status derive_geometry(const irs_params &p, int64_t n_lens, HostGeometry &out,
                           std::string &err)
{
    char buf[256];
    if (!finite_nonneg(p.kappa_star) || !finite_nonneg(p.kappa_c) || !std::isfinite(p.gamma)) {
        err = "kappa_star, kappa_c must be finite and >= 0; gamma finite";
        return IRS_E_INVALID;
    }
    if (!(std::isfinite(p.source_side) && p.source_side > 0.0)) {
        err = "source_side must be finite and > 0";
        return IRS_E_INVALID;
    }
    if (p.npix_side <= 0 || p.npix_side > 46340) {
        err = "npix_side must be in [1, 46340]";
        return IRS_E_INVALID;
    }
    if (n_lens < 0 || n_lens > (int64_t)INT32_MAX) {
        err = "n_lens must be in [0, 2^31)";
        return IRS_E_INVALID;
    }
    if (p.method != IRS_DIRECT && p.method != IRS_INTERP && p.method != IRS_LEARNED) {
        err = "method must be IRS_DIRECT, IRS_INTERP or IRS_LEARNED";
        return IRS_E_UNSUPPORTED;
    }
    if (p.precision != IRS_FP64 && p.precision != IRS_FP32_KAHAN) {
        err = "precision must be IRS_FP64 or IRS_FP32_KAHAN";
        return IRS_E_UNSUPPORTED;
    }
    const bool circle = (p.flags & IRS_CIRCLE) != 0;
    if (circle && (p.method != IRS_DIRECT || p.precision != IRS_FP64)) {
        // the level-1 grid (interpolation, FP32 near-lens residuals) tiles the
        // rectangle, not the circle around it
        err = "the circular lens plane (IRS_CIRCLE) is supported by the direct method in FP64 only";
        return IRS_E_UNSUPPORTED;
    }
    const double kappa = p.kappa_star + p.kappa_c;
    const double lam_x = 1.0 - kappa - p.gamma;   // macro eigenvalue along theta_1
    const double lam_y = 1.0 - kappa + p.gamma;   // macro eigenvalue along theta_2
    const double eps = p.crit_eps > 0.0 ? p.crit_eps : 1e-3;
    if (std::fabs(lam_x) < eps || std::fabs(lam_y) < eps) {
        std::snprintf(buf, sizeof buf,
                      "critical line: |1-kappa-gamma| = %.3g, |1-kappa+gamma| = %.3g (< %.3g)",
                      std::fabs(lam_x), std::fabs(lam_y), eps);
        err = buf;
        return IRS_E_CRITICAL;
    }
    const double border = p.border >= 0.0 ? p.border : 10.0 * std::sqrt(p.kappa_star);
    const double side = p.source_side + 2.0 * border;
    const double ix = side / std::fabs(lam_x);
    const double iy = side / std::fabs(lam_y);

    int64_t n_rays = p.n_rays;
    if (n_rays <= 0) {
        if (!(std::isfinite(p.rays_per_pixel) && p.rays_per_pixel > 0.0)) {
            err = "rays_per_pixel must be > 0 when n_rays <= 0";
            return IRS_E_INVALID;
        }
        n_rays = round_half_up(p.rays_per_pixel * (double)p.npix_side * (double)p.npix_side);
    }
    if (n_rays <= 0) {
        err = "no rays";
        return IRS_E_INVALID;
    }
    const double dx3 = std::sqrt(ix * iy / (double)n_rays);
    int64_t nx = round_half_up(ix / dx3), ny = round_half_up(iy / dx3);
    if (nx < 1) nx = 1;
    if (ny < 1) ny = 1;
    if (nx >= ((int64_t)1 << 31) || ny >= ((int64_t)1 << 31)) {
        err = "ray grid too large (nx, ny must stay below 2^31)";
        return IRS_E_INVALID;
    }

    const double short_side = std::fmin(ix, iy) / 10.0;
    const double dx1 = n_lens > 0 ? std::fmin(std::sqrt(ix * iy / (double)n_lens), short_side)
                                  : short_side;
    int64_t n1x = (int64_t)std::ceil(ix / dx1 - 1e-9);
    int64_t n1y = (int64_t)std::ceil(iy / dx1 - 1e-9);
    if (n1x < 1) n1x = 1;
    if (n1y < 1) n1y = 1;
    double dx2;
    if (p.level2_spacing > 0.0) dx2 = p.level2_spacing;
    else if (p.level2_ray_multiple > 0.0) dx2 = p.level2_ray_multiple * dx3;
    else dx2 = dx1 / 20.0;
    int64_t q = round_half_up(dx1 / dx2);
    if (q < 1) q = 1;
    if (q > 256) {
        err = "level-2 grid finer than 256 points per level-1 cell side";
        return IRS_E_INVALID;
    }
    if (p.method != IRS_DIRECT && dx1 > 1e24) {
        // the level-3 kernel takes products of four squared lens-ray distances
        // (at most 18 dx1^2 each) and needs them far from overflow
        err = "level-1 cells wider than 1e24: the interpolation needs narrower cells";
        return IRS_E_INVALID;
    }

    irs_geometry_info &g = out.info;
    g.kappa = kappa;
    g.border = border;
    g.ix = ix;
    g.iy = iy;
    g.a1 = -0.5 * ix;
    g.a2 = 0.5 * ix;
    g.b1 = -0.5 * iy;
    g.b2 = 0.5 * iy;
    g.n_rays_target = n_rays;
    g.dx3 = dx3;
    g.nx = nx;
    g.ny = ny;
    g.ray_dx = ix / (double)nx;
    g.ray_dy = iy / (double)ny;
    g.n_lens = n_lens;
    g.dx1 = dx1;
    g.n1x = n1x;
    g.n1y = n1y;
    g.dx2 = dx2;
    g.q = q;
    g.dpix = p.source_side / (double)p.npix_side;
    g.s_img = g.ray_dx * g.ray_dy;
    g.s_src = g.dpix * g.dpix;
    g.mu_th = 1.0 / (lam_x * lam_y);
    g.lens_radius = circle ? 0.5 * std::sqrt(ix * ix + iy * iy) : 0.0;
    // lenses at density kappa_*/pi (unit mean mass) over the lens plane
    g.n_stars_expected = circle ? round_half_up(p.kappa_star * g.lens_radius * g.lens_radius)
                                : round_half_up(p.kappa_star * ix * iy / M_PI);
    out.kappa_star = p.kappa_star;
    out.kappa_c = p.kappa_c;
    out.gamma = p.gamma;
    out.source_side = p.source_side;
    out.npix = p.npix_side;
    out.sheet = (p.flags & IRS_SHEET_OFF) == 0;
    out.circle = circle;
    return IRS_OK;
}

void level1_span(const irs_geometry_info &g, int axis, int64_t c, int64_t &first, int64_t &last)
{
    const int64_t n = axis ? g.ny : g.nx;
    const int64_t M = (axis ? g.n1y : g.n1x) * g.q;
    // first ray index whose level-2 index is >= G
    auto first_at = [&](int64_t G) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (((2 * mid + 1) * M) / (2 * n) >= G) hi = mid;
            else lo = mid + 1;
        }
        return lo;
    };
    first = first_at(c * g.q);
    last = first_at((c + 1) * g.q);
}

irs_status source_side_for_lens_count(const irs_params &p, int64_t n_star, double &side,
                                      std::string &err)
{
    irs_params t = p;
    t.npix_side = 16;
    t.n_rays = 1;
    HostGeometry hg;
    auto count = [&](double s, int64_t &n) {
        t.source_side = s;
        const irs_status st = derive_geometry(t, 0, hg, err);
        n = hg.info.n_stars_expected;
        return st;
    };
    double lo = 1e-3, hi = 1.0;
    int64_t n = 0;
    irs_status st;
    for (;;) {
        if ((st = count(hi, n)) != IRS_OK) return st;
        if (n >= n_star) break;
        hi *= 2.0;
        if (hi > 1e12) {
            err = "no source side holds that many lenses";
            return IRS_E_INVALID;
        }
    }
    for (int it = 0; it < 80; ++it) {
        const double mid = 0.5 * (lo + hi);
        if ((st = count(mid, n)) != IRS_OK) return st;
        if (n < n_star) lo = mid;
        else hi = mid;
    }
    side = hi;
    return IRS_OK;
}

}  // namespace irs
