// Device-side helpers shared by the ray-shooting kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace irs {

// Geometry as the kernels see it; filled on the host from the plan.
struct DevGeom {
    double a1, a2, b1, b2;      // lens/image rectangle
    double ray_dx, ray_dy;      // ray spacing (rays at cell centres)
    int64_t nx, ny;             // ray grid
    double kappa_star;          // sheet density
    double kpg, kmg;            // kappa + gamma, kappa - gamma (macro term, Eq. 6)
    double half_side, dpix;     // S/2 and S/npix: map [-S/2, S/2)^2
    int32_t npix;               // pixels per side
    int32_t sheet;              // 0: no sheet; 1: the rectangle's (Appendix A); 2: circle's
    int32_t n1x, n1y;           // level-1 cells
    int32_t q;                  // level-2 points per level-1 cell side
    int32_t pad_;
    double w1, h1;              // level-1 cell sides (I_x/n1x, I_y/n1y)
    double w2, h2;              // level-2 subcell sides (w1/q, h1/q)
    double inv_dpix;            // npix/S
    double sheet_f;             // -kappa_*/pi: the sheet's deflection over (I1, I2)
    double npix_f;              // npix as a double
};

constexpr int kWave = 64;

// theta of ray column i / row j, rounded as a1 + (i + 1/2) dx with the
// product and the sum rounded separately (contraction into an fma is switched
// off here), so that rays sit exactly where the geometry puts them: a one-ulp
// shift of theta changes the term of a lens at distance d by ulp/d.
__device__ __forceinline__ double ray_x(const DevGeom &g, int64_t i)
{
#pragma clang fp contract(off)
    return g.a1 + ((double)i + 0.5) * g.ray_dx;
}
__device__ __forceinline__ double ray_y(const DevGeom &g, int64_t j)
{
#pragma clang fp contract(off)
    return g.b1 + ((double)j + 0.5) * g.ray_dy;
}

// Level-2 column/row of ray column i / row j: the level-2 grid splits the
// rectangle into n1x*q columns, so the ray at (i + 1/2) ray_dx lies in column
// floor((2i+1) n1x q / (2 nx)) -- exact integer arithmetic, no rounding.
__device__ __forceinline__ int64_t level2_col(const DevGeom &g, int64_t i)
{
    return ((2 * i + 1) * (int64_t)g.n1x * g.q) / (2 * g.nx);
}
__device__ __forceinline__ int64_t level2_row(const DevGeom &g, int64_t j)
{
    return ((2 * j + 1) * (int64_t)g.n1y * g.q) / (2 * g.ny);
}

// Deflection of a uniform sheet of unit density over the rectangle, times pi
// (the two closed-form integrals of Appendix A with A = 1), arranged as a sum
// over the four corners: with u = theta_1 - a, v = theta_2 - b and sign +1 at
// (a1,b1), (a2,b2) and -1 at (a2,b1), (a1,b2),
//   I1 = sum sign * [ v/2 ln(u^2+v^2) + u atan(v/u) ]
//   I2 = sum sign * [ u/2 ln(u^2+v^2) + v atan(u/v) ]
// (p atan(q/p) and p ln(.) are taken as 0 where p = 0).  The negative sheet's
// deflection is -(kappa_*/pi) (I1, I2).
// Argument of w = u + i v for the sheet's Log(z - c_k), with the cut pointing
// away from the rectangle: up from a top corner (result in (-3 pi/2, pi/2]),
// down from a bottom corner (in (-pi/2, 3 pi/2]).  Inside the rectangle this
// is the principal argument; points on an edge, or a rounding step outside
// it, continue the interior values instead of crossing the principal cut,
// which runs along the top and bottom edges.
__device__ __forceinline__ double log_arg(double u, double v, bool top)
{
    double th = atan2(v, u);
    if (top && th > 0.5 * M_PI) th -= 2.0 * M_PI;
    if (!top && th < -0.5 * M_PI) th += 2.0 * M_PI;
    return th;
}

// corner c's signed terms of I1 and I2 (corners (a1,b1) (a2,b1) (a2,b2) (a1,b2))
__device__ __forceinline__ void sheet_unit_corner(const DevGeom &g, double t1, double t2, int c,
                                                  double &p1, double &p2)
{
    const double a = (c == 0 || c == 3) ? g.a1 : g.a2;
    const double b = (c < 2) ? g.b1 : g.b2;
    const double sgn = (c == 0 || c == 2) ? 1.0 : -1.0;
    const double u = t1 - a, v = t2 - b;
    const double lr = log(u * u + v * v);
    const double tu = (u != 0.0) ? u * atan(v / u) : 0.0;
    const double tv = (v != 0.0) ? v * atan(u / v) : 0.0;
    const double lv = (v != 0.0) ? 0.5 * v * lr : 0.0;
    const double lu = (u != 0.0) ? 0.5 * u * lr : 0.0;
    p1 = sgn * (lv + tu);
    p2 = sgn * (lu + tv);
}

__device__ __forceinline__ void sheet_unit(const DevGeom &g, double t1, double t2,
                                           double &I1, double &I2)
{
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double p1, p2;
        sheet_unit_corner(g, t1, t2, c, p1, p2);
        s1 += p1;
        s2 += p2;
    }
    I1 = s1;
    I2 = s2;
}

// floor(xs / dpix) for xs = b + S/2, with the quotient rounded as an IEEE
// division: the product by 1/dpix is within 1e-9 of that quotient for
// |quotient| < 1e6, so its floor is the same unless it lies that close to an
// integer, where the division itself decides.  For |quotient| >= 1e6 the
// result may differ from that floor by one, which lies off every map
// (npix <= 46340) either way.
__device__ __forceinline__ double pixel_floor_shifted(const DevGeom &g, double xs)
{
    const double q = xs * g.inv_dpix;
    const double f = floor(q);
    if (fabs((q - f) - 0.5) > 0.5 - 1e-9) return floor(xs / g.dpix);
    return f;
}

// Source pixel column and row of beta from (beta_1 + S/2, beta_2 + S/2);
// false (and -1, -1) off the map.
__device__ __forceinline__ bool pixel_xy_shifted(const DevGeom &g, double xs1, double xs2,
                                                 int32_t &ix, int32_t &iy)
{
    const double fx = pixel_floor_shifted(g, xs1);
    const double fy = pixel_floor_shifted(g, xs2);
    const double n = (double)g.npix;
    const bool in = fx >= 0.0 && fx < n && fy >= 0.0 && fy < n;
    ix = in ? (int32_t)fx : -1;
    iy = in ? (int32_t)fy : -1;
    return in;
}

// Source pixel of beta, -1 off the map.
__device__ __forceinline__ int32_t pixel_of(const DevGeom &g, double b1, double b2)
{
    const double fx = floor((b1 + g.half_side) / g.dpix);
    const double fy = floor((b2 + g.half_side) / g.dpix);
    const double n = (double)g.npix;
    if (!(fx >= 0.0 && fx < n && fy >= 0.0 && fy < n)) return -1;
    return (int32_t)fy * g.npix + (int32_t)fx;
}

// Rays binned by a call are counted in kLandedSlots counters (a workgroup adds
// to slot blockIdx mod kLandedSlots; the host sums them): one counter shared by
// every workgroup serialises its atomics in one L2 channel.
constexpr int kLandedSlots = 256;

__device__ __forceinline__ void landed_add(unsigned long long *landed, unsigned long long v)
{
    atomicAdd(landed + (blockIdx.x & (kLandedSlots - 1)), v);
}

// Wavefront-aggregated histogram update: lanes hitting the same pixel are
// merged (ballot on the leader's pixel) and one lane issues a single atomic
// with the group's count.  Must be called by every lane of the wave
// (pix = -1 for lanes with nothing to add).
__device__ __forceinline__ void bin_wave(uint32_t *__restrict__ counts, int32_t pix)
{
    uint64_t todo = __ballot(pix >= 0);
    const int lane = (int)__lane_id();
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int32_t lp = __shfl(pix, leader);
        const uint64_t same = __ballot(pix == lp) & todo;
        if (lane == leader) atomicAdd(&counts[lp], (uint32_t)__popcll(same));
        todo &= ~same;
    }
}

// Histogram update by runs: the wave's lanes hold consecutive rays of one
// row, which mostly share a pixel with their neighbours; each run of equal
// pixels in lane order adds its length once, from its last lane.  A pixel the
// wave meets in several runs gets several adds.  Must be called by every lane
// of the wave (pix = -1 for lanes with nothing to add).
__device__ __forceinline__ void bin_runs(uint32_t *__restrict__ counts, int32_t pix)
{
    const int lane = (int)__lane_id();
    const int32_t prev = __shfl_up(pix, 1);                 // lane 0 gets its own
    const uint64_t starts = __ballot(lane == 0 || pix != prev);
    const bool last = lane == 63 || ((starts >> (lane + 1)) & 1ull);
    if (last && pix >= 0) {
        const uint64_t upto = starts & (~0ull >> (63 - lane));  // run starts at or below
        const int first = 63 - __clzll((long long)upto);
        atomicAdd(&counts[pix], (uint32_t)(lane - first + 1));
    }
}

}  // namespace irs
