// Three-level-grid interpolation (Sec. 2.4 and its flow chart).
//
// Level 1: lenses are packed into n1x x n1y cells (k_level1.hip).  For a ray
// or level-2 point in cell (cx, cy) the lenses of the 3 x 3 block of cells
// around it are "nearby", all others "distant".
//
// Level 2 (k_level2): every level-1 cell is split into q x q subcells whose
// centres are the level-2 points.  At each point z0 the distant lenses give,
// in complex notation (z = theta_1 + i theta_2, conj(alpha) = m/(z - z_i) for
// one lens),
//     c_k = sum_far m_i (-1)^k / (z0 - z_i)^(k+1),   k = 0..4,
// the Taylor coefficients of conj(alpha_far)(z0 + h) = sum_k c_k h^k up to
// fourth order ("eight Taylor coefficients" = Re/Im of c_1..c_4).  The
// negative sheet is added in the same step: with F = (I1 - i I2)/pi its
// conjugated deflection is -kappa_* F(z), and inside the rectangle
// F = conj(z) + G(z) with G analytic,
//     G'(z)    = 1 - (i/pi) sum_k s_k Log(z - c_k),
//     G^(n)(z) = -(i/pi) sum_k s_k (-1)^n (n-2)! / (z - c_k)^(n-1),  n >= 2,
// over the corners c_k = (a1,b1), (a2,b1), (a2,b2), (a1,b2), s_k = +,-,+,-.
// So C_0 = c_0 - kappa_* F(z0), C_k = c_k - kappa_* G^(k)(z0)/k!, and the
// remaining sheet term -kappa_* conj(h) is exactly linear.  The four corner
// cells store c_k only (G is singular at the corners); their rays evaluate
// the sheet in closed form.  Everything in FP64.  k_level2 sums every distant
// lens at every point, as the paper does (IRS_LEVEL2_PAPER); the default
// path gets the same c_k, to rounding, from a three-level expansion of the
// distant field (k_super_expand, k_level2_near, k_level2_points below).
//
// Level 3 (k_level3): for every ray, conj(alpha_far + alpha_sheet) =
// C_0 + C_1 h + ... + C_4 h^4 - kappa_* conj(h) (Horner), plus the nearby
// lenses summed exactly in FP64, plus the macro term; then beta and the pixel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "level2.hpp"

namespace irs {

namespace {

constexpr int kThreads = 256;
constexpr int kL2Lens = 256;    // lenses per LDS stage
constexpr int kL2PPT = 2;       // level-2 points per lane per pass

__device__ __forceinline__ bool corner_cell(const DevGeom &g, int64_t cx, int64_t cy)
{
    return (cx == 0 || cx == g.n1x - 1) && (cy == 0 || cy == g.n1y - 1);
}

// level-2 point of column gx / row gy: centre of its subcell (no contraction)
__device__ __forceinline__ double level2_x(const DevGeom &g, int64_t gx)
{
#pragma clang fp contract(off)
    return g.a1 + ((double)gx + 0.5) * g.w2;
}
__device__ __forceinline__ double level2_y(const DevGeom &g, int64_t gy)
{
#pragma clang fp contract(off)
    return g.b1 + ((double)gy + 0.5) * g.h2;
}

struct cplx {
    double r, i;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b)
{
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}

// Sheet part of the level-2 coefficients at z0 (non-corner cells):
// out[k] = -kappa_* g_k, g_0 = F(z0), g_k = G^(k)(z0)/k!.
__device__ void sheet_coeffs(const DevGeom &g, double x0, double y0, cplx out[5])
{
    double I1, I2;
    sheet_unit(g, x0, y0, I1, I2);
    const double ipi = 1.0 / M_PI;
    cplx gk[5];
    gk[0] = {I1 * ipi, -I2 * ipi};
    double lr = 0.0, li = 0.0;          // sum s_k Log(z0 - c_k)
    cplx y2 = {0, 0}, y3 = {0, 0}, y4 = {0, 0};   // sum s_k (-1)^n (n-2)!/(z0-c_k)^(n-1)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double a = (c == 0 || c == 3) ? g.a1 : g.a2;
        const double b = (c < 2) ? g.b1 : g.b2;
        const double sgn = (c == 0 || c == 2) ? 1.0 : -1.0;
        const double u = x0 - a, v = y0 - b;
        const double d2 = u * u + v * v;
        lr += sgn * 0.5 * log(d2);
        li += sgn * log_arg(u, v, c >= 2);
        const cplx w = {u / d2, -v / d2};        // 1/(z0 - c)
        const cplx w2 = cmul(w, w), w3 = cmul(w2, w);
        y2.r += sgn * w.r;          y2.i += sgn * w.i;            // n = 2: +0!/(z-c)
        y3.r -= sgn * w2.r;         y3.i -= sgn * w2.i;           // n = 3: -1!/(z-c)^2
        y4.r += sgn * 2.0 * w3.r;   y4.i += sgn * 2.0 * w3.i;     // n = 4: +2!/(z-c)^3
    }
    // -(i/pi) (X + iY) = (Y - i X)/pi
    gk[1] = {1.0 + li * ipi, -lr * ipi};
    gk[2] = {y2.i * ipi / 2.0, -y2.r * ipi / 2.0};
    gk[3] = {y3.i * ipi / 6.0, -y3.r * ipi / 6.0};
    gk[4] = {y4.i * ipi / 24.0, -y4.r * ipi / 24.0};
#pragma unroll
    for (int k = 0; k < 5; ++k) out[k] = {-g.kappa_star * gk[k].r, -g.kappa_star * gk[k].i};
}

// Cells whose level-2 points take the sheet from the cell expansion: G is
// analytic away from the rectangle's corners, so its Taylor series about the
// cell centre converges over the cell at the ratio rho = (half diagonal) /
// (distance to the nearest corner); rho <= 0.2 keeps P = 32 terms within the
// order rule (the same ratio as the lenses outside the 7 x 7 block).  Both
// the cell and the point kernels take the decision from this function.
__device__ __forceinline__ bool sheet_fold_ok(const DevGeom &g, int32_t cx, int32_t cy)
{
    if (g.sheet != 1 || corner_cell(g, cx, cy)) return false;
    const double x = g.a1 + ((double)cx + 0.5) * g.w1, y = g.b1 + ((double)cy + 0.5) * g.h1;
    const double du = fmin(x - g.a1, g.a2 - x), dv = fmin(y - g.b1, g.b2 - y);
    const double hd2 = 0.25 * (g.w1 * g.w1 + g.h1 * g.h1);
    return hd2 <= 0.04 * (du * du + dv * dv);
}

// Corner c's part of the sheet's terms 0 and 1 of a cell expansion about
// (x, y), whose sums over the four corners sheet_cell_term takes: for term 0
// the signed terms of I1, I2 (sheet_unit); for term 1 the real and
// imaginary part of s_c Log(z - c).  The logarithms and arctangents make
// these the costly terms, so the cell kernel takes one corner a lane.
__device__ __forceinline__ cplx sheet_corner_low(const DevGeom &g, double x, double y, int c,
                                                 bool term1)
{
    if (!term1) {
        double p1, p2;
        sheet_unit_corner(g, x, y, c, p1, p2);
        return {p1, p2};
    }
    const double a = (c == 0 || c == 3) ? g.a1 : g.a2;
    const double b = (c < 2) ? g.b1 : g.b2;
    const double sgn = (c == 0 || c == 2) ? 1.0 : -1.0;
    const double u = x - a, v = y - b;
    return {sgn * 0.5 * log(u * u + v * v), sgn * log_arg(u, v, c >= 2)};
}

// Term k of the sheet's part of a cell expansion about (x, y) with scale s,
// in the cell expansions' convention ((1/s) sum_k L_k u^k, u = (z - zc)/s):
// -kappa_* s^(k+1) G^(k)(zc)/k!, with G = F - conj(z), G' = 1 - (i/pi) sum_c
// s_c Log(z - c), G^(k)/k! = -(i/pi) (-1)^k/(k (k-1)) sum_c s_c/(z - c)^(k-1).
// For k = 0 and 1, q is the sum of sheet_corner_low over the four corners.
__device__ cplx sheet_cell_term(const DevGeom &g, double x, double y, double s, int k, cplx q)
{
    const double ipi = 1.0 / M_PI;
    double vr, vi;
    if (k == 0) {
        vr = (q.r * ipi - x) * s;
        vi = (-q.i * ipi + y) * s;
    } else if (k == 1) {
        const double lr = q.r, li = q.i;
        vr = (1.0 + li * ipi) * s * s;
        vi = -lr * ipi * s * s;
    } else {
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double a = (c == 0 || c == 3) ? g.a1 : g.a2;
            const double b = (c < 2) ? g.b1 : g.b2;
            const double sgn = (c == 0 || c == 2) ? 1.0 : -1.0;
            const double u = x - a, v = y - b;
            const double id = s / (u * u + v * v);
            cplx w = {u * id, -v * id};                   // s/(z - c)
            cplx pw = {1.0, 0.0};                         // w^(k-1) by squaring
            for (int e = k - 1; e > 0; e >>= 1) {
                if (e & 1) pw = cmul(pw, w);
                w = cmul(w, w);
            }
            ar += sgn * pw.r;
            ai += sgn * pw.i;
        }
        const double f = ((k & 1) ? -1.0 : 1.0) / (double)(k * (k - 1)) * s * s;
        vr = f * ai * ipi;                                 // -(i/pi) f (ar + i ai)
        vi = -f * ar * ipi;
    }
    return {-g.kappa_star * vr, -g.kappa_star * vi};
}

template <bool UNIT>
__global__ __launch_bounds__(kThreads) void k_level2(
    DevGeom g, const double *__restrict__ lx, const double *__restrict__ ly,
    const double *__restrict__ lm, const int32_t *__restrict__ cell_start, int32_t nl,
    int32_t cy0, double *__restrict__ coef)
{
    __shared__ double s_x[kL2Lens], s_y[kL2Lens], s_m[UNIT ? 1 : kL2Lens];
    const int tid = threadIdx.x;
    const int32_t cx = (int32_t)(blockIdx.x % (uint32_t)g.n1x);
    const int32_t cy = cy0 + (int32_t)(blockIdx.x / (uint32_t)g.n1x);
    const int q = g.q;
    const int npts = q * q;

    // distant lenses = complement of the 3 x 3 block: at most 4 sorted ranges
    int32_t rb[4], re[4];
    int nr = 0;
    {
        int32_t prev = 0;
        const int32_t xl = cx > 0 ? cx - 1 : 0, xh = cx < g.n1x - 1 ? cx + 1 : g.n1x - 1;
        const int32_t yl = cy > 0 ? cy - 1 : 0, yh = cy < g.n1y - 1 ? cy + 1 : g.n1y - 1;
        for (int32_t row = yl; row <= yh; ++row) {
            const int32_t nb = cell_start[row * g.n1x + xl];
            const int32_t ne = cell_start[row * g.n1x + xh + 1];
            if (nb > prev) { rb[nr] = prev; re[nr] = nb; ++nr; }
            prev = ne;
        }
        if (prev < nl) { rb[nr] = prev; re[nr] = nl; ++nr; }
    }
    const bool corner = corner_cell(g, cx, cy);
    const int64_t nxq = (int64_t)g.n1x * q;

    for (int p0 = 0; p0 < npts; p0 += kThreads * kL2PPT) {
        double zr[kL2PPT], zi[kL2PPT];
        cplx c[kL2PPT][5];
#pragma unroll
        for (int k = 0; k < kL2PPT; ++k) {
            const int pt = min(p0 + tid + k * kThreads, npts - 1);
            zr[k] = level2_x(g, (int64_t)cx * q + pt % q);
            zi[k] = level2_y(g, (int64_t)cy * q + pt / q);
#pragma unroll
            for (int o = 0; o < 5; ++o) c[k][o] = {0.0, 0.0};
        }
        for (int rg = 0; rg < nr; ++rg) {
            for (int32_t base = rb[rg]; base < re[rg]; base += kL2Lens) {
                __syncthreads();
                if (base + tid < re[rg]) {
                    s_x[tid] = lx[base + tid];
                    s_y[tid] = ly[base + tid];
                    if (!UNIT) s_m[tid] = lm[base + tid];
                }
                __syncthreads();
                const int cnt = min(kL2Lens, re[rg] - base);
                for (int t = 0; t < cnt; ++t) {
                    const double X = s_x[t], Y = s_y[t];
                    const double M = UNIT ? 1.0 : s_m[t];
#pragma unroll
                    for (int k = 0; k < kL2PPT; ++k) {
                        const double wr = zr[k] - X, wi = zi[k] - Y;
                        const double inv = 1.0 / (wr * wr + wi * wi);
                        const cplx u = {wr * inv, -wi * inv};       // 1/(z0 - z_i)
                        cplx t1 = UNIT ? u : cplx{M * u.r, M * u.i};
                        c[k][0].r += t1.r; c[k][0].i += t1.i;
                        cplx t2 = cmul(t1, u);
                        c[k][1].r -= t2.r; c[k][1].i -= t2.i;
                        cplx t3 = cmul(t2, u);
                        c[k][2].r += t3.r; c[k][2].i += t3.i;
                        cplx t4 = cmul(t3, u);
                        c[k][3].r -= t4.r; c[k][3].i -= t4.i;
                        cplx t5 = cmul(t4, u);
                        c[k][4].r += t5.r; c[k][4].i += t5.i;
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kL2PPT; ++k) {
            const int pt = p0 + tid + k * kThreads;
            if (pt >= npts) continue;
            if (g.sheet && !corner) {
                cplx sh[5];
                sheet_coeffs(g, zr[k], zi[k], sh);
#pragma unroll
                for (int o = 0; o < 5; ++o) { c[k][o].r += sh[o].r; c[k][o].i += sh[o].i; }
            }
            const int64_t gx = (int64_t)cx * q + pt % q;
            const int64_t gyb = (int64_t)(cy - cy0) * q + pt / q;
            double *dst = coef + (gyb * nxq + gx) * 10;
#pragma unroll
            for (int o = 0; o < 5; ++o) {
                dst[2 * o] = c[k][o].r;
                dst[2 * o + 1] = c[k][o].i;
            }
        }
    }
}

// -------------------------------------------------------------------------
// Level 2 through one local expansion per level-1 cell.
//
// For a cell with centre zc the distant lenses split into the ring (inside the
// (2R+1) x (2R+1) block of cells around it, outside the 3 x 3 block) and the
// rest.  The rest are summed once per cell into the expansion
//     sum_i m_i / (z - z_i) = (1/s) sum_{n<P} Lt_n ((z - zc)/s)^n,
//     Lt_n = sum_i m_i (-1)^n (s/(zc - z_i))^(n+1),       s = cell scale,
// which converges at every point of the cell with ratio <= rho = (half cell
// diagonal)/((R + 1/2) * shortest cell side); the library picks P so that the
// truncation stays below ~1e-15 relative.  Each level-2 point z0 then takes
//     c_k = (1/s^(k+1)) sum_{n>=k} C(n,k) Lt_n ((z0 - zc)/s)^(n-k)
// plus the ring lenses summed directly with the c_k formula.  The result is the
// same c_k as the per-point sum over all distant lenses, to FP64 rounding.
//
// One workgroup = four cells of one level-1 row (one wave per cell).  Lens
// tiles are staged in LDS once for the four waves; each lane takes four lenses
// of a tile.  The expansions are combined across lanes by a reduce-scatter.
// -------------------------------------------------------------------------
constexpr int kCellsPerBlock = kThreads / kWave;

// 1/d for d > 0: hardware reciprocal estimate refined by two Newton steps
// (error ~1 ulp; the IEEE division sequence is not needed here)
__device__ __forceinline__ double rcp64(double d)
{
    double v = __builtin_amdgcn_rcp(d);
    double e = fma(-d, v, 1.0);
    v = fma(v, e, v);
    e = fma(-d, v, 1.0);
    return fma(v, e, v);
}

// Whole-wave reduce-scatter (every lane active): each lane holds v[0..N), N a
// multiple of 64; afterwards lane L holds in v[0..N/64) the sums over the 64
// lanes of entries L N/64 .. L N/64 + N/64 - 1.  Six halving steps: in the step
// of lane bit b the lane keeps the lower half of its list if b is clear, the
// upper half if set, and adds the partner's copy of that half (the partner
// differs in bit b and agrees in every higher bit).  Bits 5 and 4 exchange
// through gfx950's half-wave and row swaps, bits 3 .. 0 through DPP (row
// mirror, half-row mirror, quad permutations).  The order of the additions is
// fixed, so the sums are reproducible.
__device__ __forceinline__ uint32_t lo32(double v) { return (uint32_t)__double_as_longlong(v); }
__device__ __forceinline__ uint32_t hi32(double v) { return (uint32_t)((uint64_t)__double_as_longlong(v) >> 32); }
__device__ __forceinline__ double from32(uint32_t lo, uint32_t hi)
{
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// one DPP halving step: H entries kept of 2H, partner lane by DPP control C
template <int C, int H, int N>
__device__ __forceinline__ void dpp_half(double (&v)[N], bool up)
{
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const double keep = up ? v[i + H] : v[i];
        const double send = up ? v[i] : v[i + H];
        const uint32_t rl = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lo32(send), C, 0xf, 0xf, false);
        const uint32_t rh = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)hi32(send), C, 0xf, 0xf, false);
        v[i] = keep + from32(rl, rh);
    }
}

template <int N>
__device__ __forceinline__ void wave_reduce_scatter(double (&v)[N])
{
    static_assert(N % kWave == 0, "a multiple of the wave size");
    // bit 5: lanes 0-31 keep the lower half, lanes 32-63 the upper
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
        const auto l = __builtin_amdgcn_permlane32_swap(lo32(v[i]), lo32(v[i + N / 2]), false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi32(v[i]), hi32(v[i + N / 2]), false, false);
        v[i] = from32(l[0], h[0]) + from32(l[1], h[1]);
    }
    // bit 4: rows 0 and 2 keep the lower half, rows 1 and 3 the upper
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
        const auto l = __builtin_amdgcn_permlane16_swap(lo32(v[i]), lo32(v[i + N / 4]), false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi32(v[i]), hi32(v[i + N / 4]), false, false);
        v[i] = from32(l[0], h[0]) + from32(l[1], h[1]);
    }
    // bits 3 .. 0 (row mirror: lane ^ 15, half-row mirror: lane ^ 7, quad
    // permutations: lane ^ 2, lane ^ 1)
    const int lane = (int)(threadIdx.x % kWave);
    dpp_half<0x140, N / 8>(v, (lane & 8) != 0);
    dpp_half<0x141, N / 16>(v, (lane & 4) != 0);
    dpp_half<0x4e, N / 32>(v, (lane & 2) != 0);
    dpp_half<0xb1, N / 64>(v, (lane & 1) != 0);
}

template <bool UNIT, int P>
__global__ __launch_bounds__(kThreads) void k_level2_expand(
    DevGeom g, const double *__restrict__ lx, const double *__restrict__ ly,
    const double *__restrict__ lm, const uint32_t *__restrict__ lcxy, int32_t nl, int32_t cy0,
    int32_t nxb, int32_t nchunk, int32_t chunk_len, double *__restrict__ part)
{
    __shared__ double s_x[kThreads], s_y[kThreads], s_m[UNIT ? 1 : kThreads];
    __shared__ uint32_t s_c[kThreads];

    const int tid = threadIdx.x;
    const int lane = tid % kWave, wave = tid / kWave;
    const int32_t group = (int32_t)(blockIdx.x / (uint32_t)nchunk);
    const int32_t chunk = (int32_t)(blockIdx.x % (uint32_t)nchunk);
    const int32_t cy = cy0 + group / nxb;
    const int32_t cx = (group % nxb) * kCellsPerBlock + wave;     // this wave's cell
    const bool live = cx < g.n1x;
    const double sc = fmax(g.w1, g.h1), isc = 1.0 / sc;
    const double zcr = g.a1 + ((double)cx + 0.5) * g.w1;
    const double zci = g.b1 + ((double)cy + 0.5) * g.h1;
    const int32_t lo = chunk * chunk_len;
    const int32_t hi = min(nl, lo + chunk_len);

    // partial expansion of this chunk's lenses outside the (2R+1)^2 block
    // L[2n], L[2n + 1]: real and imaginary part of term n; zero padding to NV
    constexpr int NV = (2 * P + kWave - 1) / kWave * kWave;
    double L[NV];
#pragma unroll
    for (int e = 0; e < NV; ++e) L[e] = 0.0;
    // each thread's lens of the next stage is loaded while this stage is summed
    double fx = 0.0, fy = 0.0, fm = 0.0;
    uint32_t fc = 0u;
    if (lo + tid < hi) {
        fx = lx[lo + tid];
        fy = ly[lo + tid];
        if (!UNIT) fm = lm[lo + tid];
        fc = lcxy[lo + tid];
    }
    for (int32_t base = lo; base < hi; base += kThreads) {
        __syncthreads();
        if (base + tid < hi) {
            s_x[tid] = fx;
            s_y[tid] = fy;
            if (!UNIT) s_m[tid] = fm;
            s_c[tid] = fc;
        }
        __syncthreads();
        if (base + kThreads + tid < hi) {
            const int32_t li = base + kThreads + tid;
            fx = lx[li];
            fy = ly[li];
            if (!UNIT) fm = lm[li];
            fc = lcxy[li];
        }
        const int cnt = min(kThreads, hi - base);
        // two lenses per lane at a time: two independent power chains
#pragma unroll
        for (int k = 0; k < kThreads / kWave; k += 2) {
            if (k * kWave >= cnt) break;                  // the stage's lenses are done
            double tr[2], ti[2], vr[2], vi[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int t = lane + (k + e) * kWave;
                bool use = live && t < cnt;
                double X = zcr + sc, Y = zci, M = 0.0;   // harmless stand-in
                if (use) {
                    const uint32_t c = s_c[t];
                    const int32_t lcx = (int32_t)(c & 0xffffu), lcy = (int32_t)(c >> 16);
                    use = abs(lcx - cx) > kRing || abs(lcy - cy) > kRing;
                    if (use) {
                        X = s_x[t];
                        Y = s_y[t];
                        M = UNIT ? 1.0 : s_m[t];
                    }
                }
                const double wr = (zcr - X) * isc, wi = (zci - Y) * isc;
                const double inv = rcp64(wr * wr + wi * wi);
                const double ur = wr * inv, ui = -wi * inv;       // s/(zc - z_i)
                tr[e] = M * ur;                                   // m u^(n+1) (-1)^n
                ti[e] = M * ui;
                vr[e] = -ur;
                vi[e] = -ui;
            }
#pragma unroll
            for (int n = 0; n < P; ++n) {
                L[2 * n] += tr[0] + tr[1];
                L[2 * n + 1] += ti[0] + ti[1];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const double nr = tr[e] * vr[e] - ti[e] * vi[e];
                    ti[e] = tr[e] * vi[e] + ti[e] * vr[e];
                    tr[e] = nr;
                }
            }
        }
    }
    wave_reduce_scatter(L);
    if (live) {
        double *dst = part + (((int64_t)(cy - cy0) * g.n1x + cx) * nchunk + chunk) * P * 2;
#pragma unroll
        for (int r = 0; r < NV / kWave; ++r) {
            const int e = lane * (NV / kWave) + r;
            if (e < 2 * P) dst[e] = L[r];
        }
    }
}

// -------------------------------------------------------------------------
// Two-level distant field.  The distant lenses of a cell (outside its 7 x 7
// block) are those outside the (2 R_S + 1)^2 block of super cells around the
// cell's super cell (K_S x K_S level-1 cells each) plus those inside that
// block but outside the 7 x 7 block.  The former are summed once per super
// cell into an expansion of order PS about its centre zS, scale sS:
//     (1/sS) sum_n E_n u^n,  u = (z - zS)/sS,
//     E_n = sum_i m_i (-1)^n (sS/(zS - z_i))^(n+1),
// which converges over the super cell with ratio rho_S = (super half
// diagonal)/((R_S + 1/2) K_S * shortest cell side).  It is translated to each
// of its cells (re-expansion about the cell centre: with d = (zc - zS)/sS,
//     Lt_k += (s/sS)^(k+1) sum_{n>=k} C(n,k) E_n d^(n-k)),
// and the latter, at most (2 R_S + 1)^2 K_S^2 cells of lenses, are summed into
// Lt per cell directly.  The cell expansion is the same series as summing all
// distant lenses into it, to FP64 rounding; the work per cell drops from N_*
// lenses to about (2 R_S + 1)^2 K_S^2 lenses plus N_* / K_S^2, and K_S is
// chosen per plan to balance the two (super_side).
// -------------------------------------------------------------------------
constexpr int kSuperR = 2;                     // R_S (and the mid cells' block radius)
constexpr int kSuperKMax = 32;                 // largest super-cell side (cells)

// centre and scale of super cell (X, Y) of side ks cells
__device__ __forceinline__ void super_centre(const DevGeom &g, int32_t X, int32_t Y, int32_t ks,
                                             double &zr, double &zi, double &sS)
{
    zr = g.a1 + ((double)(ks * X) + 0.5 * ks) * g.w1;
    zi = g.b1 + ((double)(ks * Y) + 0.5 * ks) * g.h1;
    sS = ks * fmax(g.w1, g.h1);
}

// partial super expansions: one wave per super cell, four per workgroup,
// lenses of one chunk; part[(((Y nSx + X) nchunk + chunk) PS + n) 2 + c]
template <bool UNIT, int PS>
__global__ __launch_bounds__(kThreads) void k_super_expand(
    DevGeom g, const double *__restrict__ lx, const double *__restrict__ ly,
    const double *__restrict__ lm, const uint32_t *__restrict__ lcxy, int32_t nl, int32_t Y0,
    int32_t nSx, int32_t nSxb, int32_t nchunk, int32_t chunk_len, int32_t ks,
    double *__restrict__ part)
{
    __shared__ double s_x[kThreads], s_y[kThreads], s_m[UNIT ? 1 : kThreads];
    __shared__ uint32_t s_c[kThreads];
    const int tid = threadIdx.x;
    const int lane = tid % kWave, wave = tid / kWave;
    const int32_t group = (int32_t)(blockIdx.x / (uint32_t)nchunk);
    const int32_t chunk = (int32_t)(blockIdx.x % (uint32_t)nchunk);
    const int32_t Y = Y0 + group / nSxb;
    const int32_t X = (group % nSxb) * kCellsPerBlock + wave;
    const bool live = X < nSx;
    double zr, zi, sS;
    super_centre(g, X, Y, ks, zr, zi, sS);
    const double isc = 1.0 / sS;
    // the 5 x 5 block of super cells around (X, Y), in level-1 cells: a lens
    // in cell column c lies in super column c / ks, outside the block exactly
    // when c < (X - R_S) ks or c >= (X + R_S + 1) ks
    const int32_t ex0 = (X - kSuperR) * ks, ex1 = (X + kSuperR + 1) * ks;
    const int32_t ey0 = (Y - kSuperR) * ks, ey1 = (Y + kSuperR + 1) * ks;
    const int32_t lo = chunk * chunk_len;
    const int32_t hi = min(nl, lo + chunk_len);
    // L[2n], L[2n + 1]: real and imaginary part of term n; zero padding to NV
    constexpr int NV = (2 * PS + kWave - 1) / kWave * kWave;
    double L[NV];
#pragma unroll
    for (int e = 0; e < NV; ++e) L[e] = 0.0;
    // each thread's lens of the next stage is loaded while this stage is summed
    double fx = 0.0, fy = 0.0, fm = 0.0;
    uint32_t fc = 0u;
    if (lo + tid < hi) {
        fx = lx[lo + tid];
        fy = ly[lo + tid];
        if (!UNIT) fm = lm[lo + tid];
        fc = lcxy[lo + tid];
    }
    for (int32_t base = lo; base < hi; base += kThreads) {
        __syncthreads();
        if (base + tid < hi) {
            s_x[tid] = fx;
            s_y[tid] = fy;
            if (!UNIT) s_m[tid] = fm;
            s_c[tid] = fc;
        }
        __syncthreads();
        if (base + kThreads + tid < hi) {
            const int32_t li = base + kThreads + tid;
            fx = lx[li];
            fy = ly[li];
            if (!UNIT) fm = lm[li];
            fc = lcxy[li];
        }
        const int cnt = min(kThreads, hi - base);
#pragma unroll
        for (int k = 0; k < kThreads / kWave; k += 2) {
            if (k * kWave >= cnt) break;                  // the stage's lenses are done
            double tr[2], ti[2], vr[2], vi[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int t = lane + (k + e) * kWave;
                bool use = live && t < cnt;
                double Xl = zr + sS, Yl = zi, M = 0.0;     // harmless stand-in
                if (use) {
                    const uint32_t c = s_c[t];
                    const int32_t lcx = (int32_t)(c & 0xffffu), lcy = (int32_t)(c >> 16);
                    use = lcx < ex0 || lcx >= ex1 || lcy < ey0 || lcy >= ey1;
                    if (use) {
                        Xl = s_x[t];
                        Yl = s_y[t];
                        M = UNIT ? 1.0 : s_m[t];
                    }
                }
                const double wr = (zr - Xl) * isc, wi = (zi - Yl) * isc;
                const double inv = rcp64(wr * wr + wi * wi);
                const double ur = wr * inv, ui = -wi * inv;
                tr[e] = M * ur;
                ti[e] = M * ui;
                vr[e] = -ur;
                vi[e] = -ui;
            }
#pragma unroll
            for (int n = 0; n < PS; ++n) {
                L[2 * n] += tr[0] + tr[1];
                L[2 * n + 1] += ti[0] + ti[1];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const double nr = tr[e] * vr[e] - ti[e] * vi[e];
                    ti[e] = tr[e] * vi[e] + ti[e] * vr[e];
                    tr[e] = nr;
                }
            }
        }
    }
    wave_reduce_scatter(L);
    if (live) {
        double *dst = part + (((int64_t)(Y - Y0) * nSx + X) * nchunk + chunk) * PS * 2;
#pragma unroll
        for (int r = 0; r < NV / kWave; ++r) {
            const int e = lane * (NV / kWave) + r;
            if (e < 2 * PS) dst[e] = L[r];
        }
    }
}

// chunk partials summed in chunk order into the super table
__global__ __launch_bounds__(kThreads) void k_super_reduce(const double *__restrict__ part, int64_t n_out,
                                                           int32_t nchunk, int32_t PS,
                                                           double *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n_out) return;
    const int64_t cellterm = e / 2, comp = e % 2;
    const int64_t cell = cellterm / PS, n = cellterm % PS;
    const double *src = part + ((cell * nchunk) * PS + n) * 2 + comp;
    double acc = 0.0;
    for (int k = 0; k < nchunk; ++k) acc += src[(int64_t)k * PS * 2];
    out[e] = acc;
}

// Child expansions from a parent level: a child (a level-1 cell, kc = 1, or a
// mid cell of kc x kc cells) takes its parent's expansion (parent cells of ks
// x ks cells, PS terms about the parent's centre) re-expanded about its own
// centre, plus the lenses of the parent's 5 x 5 block that lie outside the
// child's own exclusion block (rc children each way: 7 x 7 cells for a cell,
// 5 x 5 mid cells for a mid cell), summed into P terms about its centre.
// One wave per child, four children (of one parent) per workgroup; rows of
// children from c0:  out[(((cy - c0) nCx + cx) P + n) 2 + c].
constexpr int kSuperRows = (2 * kSuperR + 1) * kSuperKMax; // cell rows of a parent block, at most

// Waves a SIMD: three for the 32-term children (168 registers and a few
// spills beat two waves without), two for the 40- and 48-term ones.
template <bool UNIT, int P, int PS>
__global__ __launch_bounds__(kThreads, P == 32 ? 3 : 2) void k_level2_near(
    DevGeom g, const double *__restrict__ lx, const double *__restrict__ ly,
    const double *__restrict__ lm, const uint32_t *__restrict__ lcxy,
    const int32_t *__restrict__ cell_start, const double *__restrict__ super, int32_t nSx,
    int32_t c0, int32_t nxb, int32_t ks, int32_t kc, int32_t rc, int32_t nCx, int32_t fold,
    double *__restrict__ out)
{
    __shared__ double s_x[kThreads], s_y[kThreads], s_m[UNIT ? 1 : kThreads];
    __shared__ uint32_t s_c[kThreads];
    __shared__ double2 s_A[kWave + PS];     // n! E_n, zero from n = PS on
    __shared__ double s_F[kWave];           // (sc/sS)^(k+1)/k!
    __shared__ int32_t s_pb[kSuperRows], s_off[kSuperRows + 1];
    const int tid = threadIdx.x;
    const int lane = tid % kWave, wave = tid / kWave;
    const int32_t cy = c0 + (int32_t)(blockIdx.x / (uint32_t)nxb);
    const int32_t cx0 = (int32_t)(blockIdx.x % (uint32_t)nxb) * kCellsPerBlock;
    const int32_t cx = cx0 + wave;
    const bool live = cx < nCx;
    // ks / kc is a multiple of kCellsPerBlock: the workgroup's children share a parent
    const int32_t X = cx0 * kc / ks, Y = cy * kc / ks;
    // the parent expansion and the lens ranges of the parent block, row by row
    for (int n = tid; n < kWave + PS; n += kThreads) {
        double2 a = {0.0, 0.0};
        if (n < PS) {
            double f = 1.0;                                   // n!
            for (int t = 2; t <= n; ++t) f *= (double)t;
            const double *src = super + (((int64_t)Y * nSx + X) * PS + n) * 2;
            a = {src[0] * f, src[1] * f};
        }
        s_A[n] = a;
    }
    const int32_t ya = max(0, (Y - kSuperR) * ks), yb = min(g.n1y, (Y + kSuperR + 1) * ks);
    const int32_t xa = max(0, (X - kSuperR) * ks), xb = min(g.n1x, (X + kSuperR + 1) * ks);
    const int nrow = yb - ya;
    if (tid < nrow) {
        const int32_t row = ya + tid;
        s_pb[tid] = cell_start[row * g.n1x + xa];
        s_off[tid + 1] = cell_start[row * g.n1x + xb] - cell_start[row * g.n1x + xa];
    }
    __syncthreads();
    const double sc = kc * fmax(g.w1, g.h1), isc = 1.0 / sc;
    // the child's exclusion block in level-1 cells (a lens in cell column c
    // lies in child column c / kc: outside the block exactly when
    // c < (cx - rc) kc or c >= (cx + rc + 1) kc)
    const int32_t ex0 = (cx - rc) * kc, ex1 = (cx + rc + 1) * kc;
    const int32_t ey0 = (cy - rc) * kc, ey1 = (cy + rc + 1) * kc;
    double zSr, zSi, sS;
    super_centre(g, X, Y, ks, zSr, zSi, sS);
    if (tid == 0) {
        s_off[0] = 0;
        for (int r = 0; r < nrow; ++r) s_off[r + 1] += s_off[r];
        const double ratio = sc / sS;
        double f = ratio;
        for (int k = 0; k < kWave; ++k) {
            s_F[k] = f;
            f *= ratio / (double)(k + 1);
        }
    }
    __syncthreads();
    const int32_t total = s_off[nrow];

    const double zcr = g.a1 + ((double)(kc * cx) + 0.5 * kc) * g.w1;
    const double zci = g.b1 + ((double)(kc * cy) + 0.5 * kc) * g.h1;

    // L[2n], L[2n + 1]: real and imaginary part of term n; zero padding to NV
    constexpr int NV = (2 * P + kWave - 1) / kWave * kWave;
    double L[NV];
#pragma unroll
    for (int e = 0; e < NV; ++e) L[e] = 0.0;
    // each thread's lens of the next stage is loaded while this stage is summed
    auto lens_of = [&](int32_t gi) {              // row of lens gi: s_off[r] <= gi < s_off[r + 1]
        int r = 0, rh = nrow - 1;
        while (r < rh) {
            const int mid = (r + rh + 1) >> 1;
            if (s_off[mid] <= gi) r = mid;
            else rh = mid - 1;
        }
        return s_pb[r] + (gi - s_off[r]);
    };
    double fx = 0.0, fy = 0.0, fm = 0.0;
    uint32_t fc = 0u;
    if (tid < total) {
        const int32_t li = lens_of(tid);
        fx = lx[li];
        fy = ly[li];
        if (!UNIT) fm = lm[li];
        fc = lcxy[li];
    }
    for (int32_t base = 0; base < total; base += kThreads) {
        __syncthreads();
        if (base + tid < total) {
            s_x[tid] = fx;
            s_y[tid] = fy;
            if (!UNIT) s_m[tid] = fm;
            s_c[tid] = fc;
        }
        __syncthreads();
        if (base + kThreads + tid < total) {
            const int32_t li = lens_of(base + kThreads + tid);
            fx = lx[li];
            fy = ly[li];
            if (!UNIT) fm = lm[li];
            fc = lcxy[li];
        }
        const int cnt = min(kThreads, total - base);
#pragma unroll
        for (int k = 0; k < kThreads / kWave; k += 2) {
            if (k * kWave >= cnt) break;                  // the stage's lenses are done
            double tr[2], ti[2], vr[2], vi[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int t = lane + (k + e) * kWave;
                bool use = live && t < cnt;
                double Xl = zcr + sc, Yl = zci, M = 0.0;   // harmless stand-in
                if (use) {
                    const uint32_t c = s_c[t];
                    const int32_t lcx = (int32_t)(c & 0xffffu), lcy = (int32_t)(c >> 16);
                    use = lcx < ex0 || lcx >= ex1 || lcy < ey0 || lcy >= ey1;
                    if (use) {
                        Xl = s_x[t];
                        Yl = s_y[t];
                        M = UNIT ? 1.0 : s_m[t];
                    }
                }
                const double wr = (zcr - Xl) * isc, wi = (zci - Yl) * isc;
                const double inv = rcp64(wr * wr + wi * wi);
                const double ur = wr * inv, ui = -wi * inv;
                tr[e] = M * ur;
                ti[e] = M * ui;
                vr[e] = -ur;
                vi[e] = -ui;
            }
#pragma unroll
            for (int n = 0; n < P; ++n) {
                L[2 * n] += tr[0] + tr[1];
                L[2 * n + 1] += ti[0] + ti[1];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const double nr = tr[e] * vr[e] - ti[e] * vi[e];
                    ti[e] = tr[e] * vi[e] + ti[e] * vr[e];
                    tr[e] = nr;
                }
            }
        }
    }
    // Translation of the parent expansion to this child, term k of
    //     T_k = (sc/sS)^(k+1) sum_(n>=k) C(n,k) E_n d^(n-k),  d = (zc - zS)/sS,
    // as F_k sum_j A_(k+j) b_j with A_n = n! E_n, b_j = d^j/j!, F_k =
    // (sc/sS)^(k+1)/k!: every lane walks the same j, so b_j is uniform.  The
    // lane computes the term whose sums it holds after the reduce-scatter
    // (with P = 32 both lanes of a term).
    constexpr int R = NV / kWave;
    const int k = R == 1 ? lane >> 1 : lane;
    double Tr, Ti;
    {
        const double dr = (zcr - zSr) / sS, di = (zci - zSi) / sS;
        double br = 1.0, bi = 0.0;
        double ar0 = 0.0, ai0 = 0.0, ar1 = 0.0, ai1 = 0.0;   // even and odd j
#pragma unroll
        for (int j = 0; j < PS; ++j) {
            const double2 a = s_A[k + j];
            if (j & 1) {
                ar1 = fma(a.x, br, fma(-a.y, bi, ar1));
                ai1 = fma(a.x, bi, fma(a.y, br, ai1));
            } else {
                ar0 = fma(a.x, br, fma(-a.y, bi, ar0));
                ai0 = fma(a.x, bi, fma(a.y, br, ai0));
            }
            const double inv = 1.0 / (double)(j + 1);
            const double nr = (br * dr - bi * di) * inv;
            bi = (br * di + bi * dr) * inv;
            br = nr;
        }
        const double f = s_F[k];
        Tr = (ar0 + ar1) * f;
        Ti = (ai0 + ai1) * f;
        if (fold && live && sheet_fold_ok(g, cx, cy)) {   // cells only, wave-uniform: the sheet's series
            // terms 0 and 1 one corner a lane (lanes 0-3: term 0, lanes 4-7:
            // term 1), summed over each group of four lanes
            cplx q = lane < 8 ? sheet_corner_low(g, zcr, zci, lane & 3, lane >= 4) : cplx{0.0, 0.0};
            q.r += __shfl_xor(q.r, 1);
            q.i += __shfl_xor(q.i, 1);
            q.r += __shfl_xor(q.r, 2);
            q.i += __shfl_xor(q.i, 2);
            const int src = k == 1 ? 4 : 0;
            q = {__shfl(q.r, src), __shfl(q.i, src)};
            if (k < P) {
                const cplx t = sheet_cell_term(g, zcr, zci, sc, k, q);
                Tr += t.r;
                Ti += t.i;
            }
        }
    }
    wave_reduce_scatter(L);
    if (live) {
        double *dst = out + ((int64_t)(cy - c0) * nCx + cx) * P * 2;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = lane * R + r;
            const double t = R == 1 ? ((lane & 1) ? Ti : Tr) : (r ? Ti : Tr);
            if (e < 2 * P) dst[e] = L[r] + t;
        }
    }
}

// Cells whose level-2 points take the sheet's closed-form coefficients: with
// the sheet, outside the corner cells, where its series is not folded into
// the cell expansion (near the rectangle's edges, or no folding at all).
__device__ __forceinline__ bool sheet_closed_form(const DevGeom &g, int32_t fold, int32_t cx,
                                                  int32_t cy)
{
    return g.sheet && !corner_cell(g, cx, cy) && !(fold && sheet_fold_ok(g, cx, cy));
}

// CLOSED = false: the cells that do not take the closed form; CLOSED = true:
// the cells that do (a workgroup with none returns at once).  The closed
// form's logarithms would otherwise set every point's register budget.
// STAGED: the ring lenses of a workgroup's four cells, which lie in one block
// of 7 rows x 10 columns of cells, are staged in LDS once; the host takes this
// instance when no such block of the plan holds more than kRingCap lenses
// (ring_fits), the other reads them from global memory.
constexpr int kRingCap = 768;
constexpr int kRingRows = 2 * kRing + 1, kRingCols = kCellsPerBlock + 2 * kRing;
// a cell's ring as runs of cells in one row: one run in each of the 2 kRing - 2
// outer rows, two (left and right of the 3 x 3 block) in each of the 3 inner
constexpr int kRingSegs = (kRingRows - 3) + 2 * 3;

template <bool UNIT, int P, bool CLOSED, bool STAGED>
__global__ __launch_bounds__(kThreads) void k_level2_points(
    DevGeom g, const double *__restrict__ lx, const double *__restrict__ ly,
    const double *__restrict__ lm, const int32_t *__restrict__ cell_start, int32_t cy0,
    int32_t nxb, int32_t nchunk, int32_t fold, const double *__restrict__ part,
    double *__restrict__ coef)
{
    __shared__ double s_L[kCellsPerBlock][P][2];
    constexpr int kCap = STAGED ? kRingCap : 1;
    __shared__ double s_rx[kCap], s_ry[kCap], s_rm[UNIT ? 1 : kCap];
    __shared__ int32_t s_cs[kRingRows][kRingCols + 1];   // cell_start over the block
    __shared__ int32_t s_rb[kRingRows + 1];              // LDS offset of each row
    __shared__ int2 s_seg[kCellsPerBlock][kRingSegs];    // STAGED: each cell's runs in LDS
    const int tid = threadIdx.x;
    const int32_t cy = cy0 + (int32_t)(blockIdx.x / (uint32_t)nxb);
    const int32_t cx0 = (int32_t)(blockIdx.x % (uint32_t)nxb) * kCellsPerBlock;
    if constexpr (CLOSED) {                                  // block-uniform
        bool any = false;
        for (int w = 0; w < kCellsPerBlock; ++w)
            any = any || (cx0 + w < g.n1x && sheet_closed_form(g, fold, cx0 + w, cy));
        if (!any) return;
    }
    const double sc = fmax(g.w1, g.h1), isc = 1.0 / sc;
    const double zci = g.b1 + ((double)cy + 0.5) * g.h1;
    // sum the chunks' partial expansions, in chunk order
    for (int e = tid; e < kCellsPerBlock * P * 2; e += kThreads) {
        const int w = e / (P * 2), n = (e / 2) % P, comp = e % 2;
        const int32_t ccx = cx0 + w;
        double acc = 0.0;
        if (ccx < g.n1x) {
            const double *src = part + (((int64_t)(cy - cy0) * g.n1x + ccx) * nchunk * P + n) * 2 + comp;
            for (int k = 0; k < nchunk; ++k) acc += src[(int64_t)k * P * 2];
        }
        s_L[w][n][comp] = acc;
    }
    // the block of cells holding every ring lens of the four cells
    const int32_t ya = max(0, cy - kRing), yb = min(g.n1y - 1, cy + kRing);
    const int32_t ua = max(0, cx0 - kRing), ub = min(g.n1x - 1, cx0 + kCellsPerBlock - 1 + kRing);
    const int nrow = yb - ya + 1, ncol = ub - ua + 1;
    for (int e = tid; e < nrow * (ncol + 1); e += kThreads) {
        const int r = e / (ncol + 1), c = e % (ncol + 1);
        s_cs[r][c] = cell_start[(int64_t)(ya + r) * g.n1x + ua + c];
    }
    __syncthreads();
    if (tid == 0) {
        s_rb[0] = 0;
        for (int r = 0; r < nrow; ++r) s_rb[r + 1] = s_rb[r] + (s_cs[r][ncol] - s_cs[r][0]);
    }
    __syncthreads();
    if constexpr (STAGED) {
        const int total = min(s_rb[nrow], kRingCap);               // == s_rb[nrow] (ring_fits)
        for (int i = tid; i < total; i += kThreads) {
            int r = 0;
            while (s_rb[r + 1] <= i) ++r;
            const int32_t src = s_cs[r][0] + (i - s_rb[r]);
            s_rx[i] = lx[src];
            s_ry[i] = ly[src];
            if (!UNIT) s_rm[i] = lm[src];
        }
        // each cell's runs of ring cells as ranges of the staged lenses, in
        // row order (rows cy - kRing .. cy + kRing; left run before right)
        if (tid < kCellsPerBlock * kRingSegs) {
            const int w = tid / kRingSegs, sg = tid % kRingSegs;
            const int outer = kRing - 1;                      // outer rows on each side
            int dr, kind;                                     // kind 0: whole, 1: left, 2: right
            if (sg < outer) { dr = sg - kRing; kind = 0; }
            else if (sg < outer + 6) { dr = (sg - outer) / 2 - 1; kind = 1 + ((sg - outer) & 1); }
            else { dr = sg - outer - 6 + 2; kind = 0; }
            const int32_t row = cy + dr, ccx = cx0 + w;
            int2 be = {0, 0};
            if (row >= ya && row <= yb && ccx < g.n1x) {
                int32_t xa = kind == 2 ? ccx + 2 : ccx - kRing;
                int32_t xb = kind == 1 ? ccx - 2 : ccx + kRing;
                xa = max(xa, 0);
                xb = min(xb, g.n1x - 1);
                if (xa <= xb) {
                    const int r = row - ya;
                    const int32_t off = s_rb[r] - s_cs[r][0];
                    be.x = min(s_cs[r][xa - ua] + off, kRingCap);
                    be.y = min(s_cs[r][xb + 1 - ua] + off, kRingCap);
                }
            }
            s_seg[w][sg] = be;
        }
    }
    __syncthreads();

    // ---- phase B: the level-2 points of the four cells
    const int q = g.q, npts = q * q;
    const int64_t nxq = (int64_t)g.n1x * q;
    for (int pp = tid; pp < kCellsPerBlock * npts; pp += kThreads) {
        const int w = pp / npts, pt = pp % npts;
        const int32_t ccx = cx0 + w;
        if (ccx >= g.n1x || sheet_closed_form(g, fold, ccx, cy) != CLOSED) continue;
        const int64_t gx = (int64_t)ccx * q + pt % q;
        const int64_t gyl = pt / q;
        const double x0 = level2_x(g, gx), y0 = level2_y(g, (int64_t)cy * q + gyl);
        const double czr = g.a1 + ((double)ccx + 0.5) * g.w1;
        const double dr = (x0 - czr) * isc, di = (y0 - zci) * isc;
        // c_k = s^-(k+1) sum_n C(n,k) Lt_n d^(n-k): the polynomial sum_n Lt_n d^n
        // and its derivatives over k! by one Horner pass from n = P-1 down
        // (D_k <- D_k d + D_(k-1), D_0 <- D_0 d + Lt_n)
        double cr[5] = {0, 0, 0, 0, 0}, ci[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int n = P - 1; n >= 0; --n) {
#pragma unroll
            for (int k = 4; k >= 0; --k) {
                const double ar = k > 0 ? cr[k - 1] : s_L[w][n][0];
                const double ai = k > 0 ? ci[k - 1] : s_L[w][n][1];
                const double nr = fma(cr[k], dr, fma(-ci[k], di, ar));
                ci[k] = fma(cr[k], di, fma(ci[k], dr, ai));
                cr[k] = nr;
            }
        }
        cplx c[5];
        double sk = isc;                                  // 1/s^(k+1)
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            c[k] = {cr[k] * sk, ci[k] * sk};
            sk *= isc;
        }
        // ring lenses: inside the (2R+1)^2 block, outside the 3 x 3 block
        auto ring_lens = [&](double X, double Y, double M) {
            const double wr = x0 - X, wi = y0 - Y;
            // 1/|w|^2: reciprocal estimate and one Newton step (~2^-48)
            const double rr = fma(wr, wr, wi * wi);
            double inv = __builtin_amdgcn_rcp(rr);
            inv = fma(inv, fma(-rr, inv, 1.0), inv);
            const cplx u = {wr * inv, -wi * inv};
            cplx t1 = UNIT ? u : cplx{M * u.r, M * u.i};
            c[0].r += t1.r; c[0].i += t1.i;
            cplx t2 = cmul(t1, u);
            c[1].r -= t2.r; c[1].i -= t2.i;
            cplx t3 = cmul(t2, u);
            c[2].r += t3.r; c[2].i += t3.i;
            cplx t4 = cmul(t3, u);
            c[3].r -= t4.r; c[3].i -= t4.i;
            cplx t5 = cmul(t4, u);
            c[4].r += t5.r; c[4].i += t5.i;
        };
        if constexpr (STAGED) {
            for (int sg = 0; sg < kRingSegs; ++sg) {
                const int2 be = s_seg[w][sg];
                for (int32_t pl = be.x; pl < be.y; ++pl) ring_lens(s_rx[pl], s_ry[pl], UNIT ? 1.0 : s_rm[pl]);
            }
        } else {
            for (int32_t row = ya; row <= yb; ++row) {
                const bool mid = abs(row - cy) <= 1;
                for (int seg = 0; seg < (mid ? 2 : 1); ++seg) {
                    int32_t xa, xb;
                    if (!mid) { xa = ccx - kRing; xb = ccx + kRing; }
                    else if (seg == 0) { xa = ccx - kRing; xb = ccx - 2; }
                    else { xa = ccx + 2; xb = ccx + kRing; }
                    xa = max(xa, 0);
                    xb = min(xb, g.n1x - 1);
                    if (xa > xb) continue;
                    const int r = row - ya;
                    const int32_t pb = s_cs[r][xa - ua], pe = s_cs[r][xb + 1 - ua];
                    for (int32_t pl = pb; pl < pe; ++pl) ring_lens(lx[pl], ly[pl], UNIT ? 1.0 : lm[pl]);
                }
            }
        }
        if (g.sheet && !corner_cell(g, ccx, cy)) {
            if constexpr (!CLOSED) {
                // G's series came with the cell expansion; F = conj(z) + G
                c[0].r -= g.kappa_star * x0;
                c[0].i += g.kappa_star * y0;
            } else {
                cplx sh[5];
                sheet_coeffs(g, x0, y0, sh);
#pragma unroll
                for (int o = 0; o < 5; ++o) { c[o].r += sh[o].r; c[o].i += sh[o].i; }
            }
        }
        double *dst = coef + (((int64_t)(cy - cy0) * q + gyl) * nxq + gx) * 10;
#pragma unroll
        for (int o = 0; o < 5; ++o) {
            dst[2 * o] = c[o].r;
            dst[2 * o + 1] = c[o].i;
        }
    }
}

// -------------------------------------------------------------------------
// Level 3: one workgroup = a 64 x 32 tile of rays (lane = column, each wave 8
// rows).  Every ray: Horner of its level-2 point's C_0..C_4, the sheet's
// linear term (closed form in corner cells), the near lenses exactly, the
// macro term, beta and the pixel.  What depends on the ray row only (theta_2,
// its level-2 and level-1 rows, the offset from the level-2 row) comes from a
// per-plan row table through scalar loads, so a wave's rows cost no vector
// work; a lane's rows share their level-2 point's coefficients until the
// level-2 row changes.  Binning: the tile's rays land in a small patch of the
// map, so the workgroup finds the bounding box of its landed pixels, counts
// into an LDS histogram over that box and flushes each non-empty bin with one
// global atomic; a box larger than the LDS histogram (rays scattered, as near
// a lens) falls back to one global add per run of equal pixels in a lane.
// -------------------------------------------------------------------------
constexpr int kL3Rows = 32;
constexpr int kXcds = 8;               // MI355X: workgroups go to the 8 XCDs in turn
constexpr int kL3RowsPerWave = kL3Rows / (kThreads / kWave);
constexpr int kHistCap = 6144;

// A level-3 workgroup's LDS: the histogram over the tile's landed-pixel box
// (row pitch a power of two) with one more bin that takes the rays it does
// not bin, the box (through LDS atomics) and the landed-ray count.
struct L3Lds {
    uint32_t hist[kHistCap + 1];
    uint32_t bmin[2];         // min x, min y of landed pixels (unsigned: -1 never wins)
    int32_t bmax[2];          // max x, max y (signed: -1 never wins)
    uint32_t landed;
};


// One ray row of the plan's ray grid, as the level-3 kernel reads it.
struct alignas(32) RowInfo {
    double t2;        // theta_2 of the row
    double hi;        // t2 minus the y of its level-2 row
    int32_t gy;       // level-2 row
    int32_t cy;       // level-1 row
    int64_t base;     // index of the row's first ray (j nx)
    double c2;        // t2 - (kappa - gamma) t2 + kappa_* hi (sheet on) + S/2
};

// floor(num / den) for 0 <= num < 2^53, den > 0, without 64-bit integer division
__device__ __forceinline__ int64_t floor_div(int64_t num, int64_t den)
{
    int64_t v = (int64_t)((double)num / (double)den);
    if (v * den > num) --v;
    else if ((v + 1) * den <= num) ++v;
    return v;
}

// Term of one nearby lens for a ray at (t1, t2): m (d1, d2)/(d1^2 + d2^2),
// d = theta - z, with d1 and d1s = d1^2 + kNearTiny taken once per lens for
// all rays of a column.  The quotient m/rr is the hardware reciprocal
// estimate v times m, corrected once (w = y + v (m - rr y)), which squares
// the estimate's relative error.  kNearTiny (far below the square of any
// lens-ray distance that occurs) keeps rr > 0 where a lens sits exactly on
// a ray, whose term is then exactly 0 because d = 0; it changes no other rr.
constexpr double kNearTiny = 1e-300;
// Largest level-1 cell side a plan may have: every nearby lens then lies
// within 3 sqrt(2) kMaxCell of a ray, so rr < 1e49 and a product of four
// rr stays below kGroupMax.
constexpr double kMaxCell = 1e24;

__device__ __forceinline__ void near_term(double d1, double d1s, double t2, double zy, double m,
                                          double &n1, double &n2)
{
    const double d2 = t2 - zy;
    const double rr = fma(d2, d2, d1s);
    const double v = __builtin_amdgcn_rcp(rr);
    const double y = m * v;
    const double w = fma(v, fma(-rr, y, m), y);
    n1 = fma(w, d1, n1);
    n2 = fma(w, d2, n2);
}

// The same for G rays of one column (rows t2s[0..G-1]): the G quotients
// m/rr_k come from one reciprocal of their product p = rr_0 ... rr_{G-1},
// corrected once as above (q = m/p), then back-substitution through the
// prefix products P_k = rr_0 ... rr_k: m/rr_k = q P_{k-1} for k = G-1 down to
// 1, q taking q rr_k = m/P_{k-1} after each step, and m/rr_0 = the last q.
// Each quotient carries at most about 2G + 4 units of rounding.  Where p lies
// at or below 1e-200 (a lens on or extremely close to a ray) the quotients are
// taken one by one, with kNearTiny added to each rr.  Cells no wider than
// kMaxCell keep p below 1e200, far from overflow, so p needs no upper test.
constexpr double kGroupMin = 1e-200;
// rows of a lane that share one reciprocal per lens: four keeps the group's
// products in few enough registers for five waves per SIMD
constexpr int kNearGroup = 4;

template <int G>
__device__ __forceinline__ void near_group_d2(double d1, double d1s, const double *d2, double m,
                                              double *n1s, double *n2s)
{
    // d1s = d1^2 here (no kNearTiny: that is added on the one-by-one path)
    double rr[G], pre[G], w[G];
#pragma unroll
    for (int k = 0; k < G; ++k) rr[k] = fma(d2[k], d2[k], d1s);
    pre[0] = rr[0];
#pragma unroll
    for (int k = 1; k < G; ++k) pre[k] = pre[k - 1] * rr[k];
    const double p = pre[G - 1];
    if (__builtin_expect(p > kGroupMin, 1)) {
        const double v = __builtin_amdgcn_rcp(p);
        const double y = m * v;
        double q = fma(v, fma(-p, y, m), y);          // m / p
#pragma unroll
        for (int k = G - 1; k >= 1; --k) {
            w[k] = q * pre[k - 1];
            q = q * rr[k];                            // m / P_{k-1}
        }
        w[0] = q;
    } else {
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const double r = rr[k] + kNearTiny;
            const double v = __builtin_amdgcn_rcp(r);
            const double y = m * v;
            w[k] = fma(v, fma(-r, y, m), y);
        }
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
        n1s[k] = fma(w[k], d1, n1s[k]);
        n2s[k] = fma(w[k], d2[k], n2s[k]);
    }
}

template <int G>
__device__ __forceinline__ void near_group(double d1, double d1s, const double *t2s, double zy,
                                           double m, double *n1s, double *n2s)
{
    double d2[G];
#pragma unroll
    for (int k = 0; k < G; ++k) d2[k] = t2s[k] - zy;
    near_group_d2<G>(d1, d1s, d2, m, n1s, n2s);
}

// Nearby lenses of RR rays in one column (t1) and RR rows (t2s) that share
// the level-1 cell row cy: the lenses of cells (xl..xh, cy-1..cy+1).  The
// loop is the same for the whole wave: it runs over the lenses of cells
// cl..ch (every lane's xl..xh lies inside, cl/ch/cy wave-uniform, so lens
// data come through scalar loads); where the wave's lanes lie in more than
// one cell column (straddle), a lane gives the lenses outside its own xl..xh
// mass 0, which adds exact zeros.  Lenses are taken in their sorted order.
// STRADDLE = false is the same pass for a wave known to lie in one column.
template <bool UNIT, int RR, bool STRADDLE>
__device__ __forceinline__ void near_pass(const DevGeom &g, const double2 *__restrict__ lxy,
                                          const double *__restrict__ lm,
                                          const int32_t *__restrict__ cell_start, int32_t cy,
                                          int32_t cl, int32_t ch, bool straddle, int32_t xl,
                                          int32_t xh, double t1, const double *t2s, double *n1s,
                                          double *n2s)
{
    const int32_t yl = cy > 0 ? cy - 1 : 0, yh = cy < g.n1y - 1 ? cy + 1 : g.n1y - 1;
    for (int32_t row = yl; row <= yh; ++row) {
        const int32_t pb = cell_start[row * g.n1x + cl];
        const int32_t pe = cell_start[row * g.n1x + ch + 1];
        int32_t lpb = pb, lpe = pe;
        if (STRADDLE && straddle) {
            lpb = cell_start[row * g.n1x + xl];
            lpe = cell_start[row * g.n1x + xh + 1];
        }
        for (int32_t q_ = pb; q_ < pe; ++q_) {
            const double2 z = lxy[q_];
            double m = UNIT ? 1.0 : lm[q_];
            if (STRADDLE && straddle) m = (q_ >= lpb && q_ < lpe) ? m : 0.0;
            const double d1 = t1 - z.x;
            if constexpr (RR > 1) {
                const double d1s = d1 * d1;
                static_assert(RR % kNearGroup == 0, "rows in whole groups");
#pragma unroll
                for (int h = 0; h < RR; h += kNearGroup)
                    near_group<kNearGroup>(d1, d1s, t2s + h, z.y, m, n1s + h, n2s + h);
            } else {
                const double d1s = fma(d1, d1, kNearTiny);
#pragma unroll
                for (int k = 0; k < RR; ++k) near_term(d1, d1s, t2s[k], z.y, m, n1s[k], n2s[k]);
            }
        }
    }
}

// Reductions over each row of 16 lanes (every lane active): four DPP row
// shifts, after which lane 15 of a row holds the row's result.  Lanes that
// a shift leaves without a source keep the identity.
constexpr int kDppRowShr = 0x110;   // row_shr:n is kDppRowShr + n
template <int N>
__device__ __forceinline__ uint32_t shr_min_u(uint32_t v)
{
    return min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)UINT32_MAX, (int)v, kDppRowShr + N,
                                                        0xf, 0xf, false));
}
template <int N>
__device__ __forceinline__ int shr_max(int v)
{
    return max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, kDppRowShr + N, 0xf, 0xf, false));
}
__device__ __forceinline__ uint32_t row_min_u(uint32_t v)
{
    return shr_min_u<8>(shr_min_u<4>(shr_min_u<2>(shr_min_u<1>(v))));
}
__device__ __forceinline__ int row_max(int v)
{
    return shr_max<8>(shr_max<4>(shr_max<2>(shr_max<1>(v))));
}

// One ray column of the plan's ray grid, as the level-3 kernel reads it: what
// takes 64-bit integer division to find (16 bytes, so that one XCD's share of
// the table stays in its L2 from one tile row to the next).
struct alignas(16) ColInfo {
    double hr;        // theta_1 minus the x of the column's level-2 column
    uint32_t coff;    // byte offset of the column's level-2 point in a level-2 row
    int32_t cx;       // level-1 column
};
static_assert(sizeof(ColInfo) == 16, "one 16-byte load a lane");

// theta_1 of ray column i < 2^31, rounded as ray_x rounds it
__device__ __forceinline__ double ray_x32(const DevGeom &g, int32_t i)
{
#pragma clang fp contract(off)
    return g.a1 + ((double)i + 0.5) * g.ray_dx;
}

// beta_1 + S/2 of a column's rays without the lens terms: the macro term and
// the sheet's -kappa_* conj(h) part (s1 = kappa_* hr; the row's c2 holds the
// same for beta_2)
__device__ __forceinline__ void column_terms(const DevGeom &g, double t1, double hr, double &c1,
                                             double &s1)
{
    s1 = g.sheet ? g.kappa_star * hr : 0.0;
    const double mac1 = g.kpg * t1;
    c1 = ((t1 - mac1) + s1) + g.half_side;
}

__global__ __launch_bounds__(kThreads) void k_col_table(DevGeom g, ColInfo *cols)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= g.nx) return;
    const int64_t nxq = (int64_t)g.n1x * g.q;
    const int64_t gx = floor_div((2 * i + 1) * nxq, 2 * g.nx);
    ColInfo c;
    c.hr = ray_x(g, i) - level2_x(g, gx);
    c.coff = (uint32_t)gx * 10u * (uint32_t)sizeof(double);
    c.cx = (int32_t)(gx / g.q);
    cols[i] = c;
}

__global__ __launch_bounds__(kThreads) void k_row_table(DevGeom g, RowInfo *rows)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= g.ny) return;
    const int64_t gy = floor_div((2 * j + 1) * (int64_t)g.n1y * g.q, 2 * g.ny);
    RowInfo r;
    r.t2 = ray_y(g, j);
    r.hi = r.t2 - level2_y(g, gy);
    r.gy = (int32_t)gy;
    r.cy = (int32_t)(gy / g.q);
    r.base = j * g.nx;
    const double mac = g.kmg * r.t2;
    const double sh = g.sheet ? g.kappa_star * r.hi : 0.0;
    r.c2 = ((r.t2 - mac) + sh) + g.half_side;
    rows[j] = r;
}

// The sheet's deflection in the rectangle's corner cells, in closed form
// minus the -kappa_* conj(h) part the column and row constants hold: the
// correction to add to (Re A, Im A).
struct D2 {
    double x, y;
};

__device__ __forceinline__ D2 corner_sheet(const DevGeom &g, double t1, double t2, double hr,
                                         double hi)
{
    double I1, I2;
    sheet_unit(g, t1, t2, I1, I2);
    return D2{g.sheet_f * I1 + g.kappa_star * hr, -(g.sheet_f * I2 + g.kappa_star * hi)};
}

// Pixel column and row of beta from (beta_1 + S/2, beta_2 + S/2): the floor
// of the products by 1/dpix, or, where either product lies within 1e-9 of an
// integer, of the IEEE quotients by dpix for both (pixel_floor_shifted's
// rule, one branch for the pair); (-1, -1) off the map.  The floor is taken
// as the nearest integer to the product minus 1/2 (one fused multiply-add),
// whose distance from that integer is the edge test.
__device__ __forceinline__ void pixel_pair(const DevGeom &g, double xs1, double xs2, int32_t &ix,
                                           int32_t &iy)
{
    const double m1 = fma(xs1, g.inv_dpix, -0.5), m2 = fma(xs2, g.inv_dpix, -0.5);
    double f1 = rint(m1), f2 = rint(m2);
    constexpr double lim = 0.5 - 1e-9;
    if ((int)(fabs(m1 - f1) > lim) | (int)(fabs(m2 - f2) > lim)) {
        f1 = floor(xs1 / g.dpix);
        f2 = floor(xs2 / g.dpix);
    }
    // the hardware conversion saturates (a value beyond the int32 range gives
    // INT32_MIN or INT32_MAX; no NaN arises here), which a C++ cast does not
    // promise: a floor off the map stays off it as an unsigned index >= npix
    int32_t jx, jy;
    asm("v_cvt_i32_f64 %0, %1" : "=v"(jx) : "v"(f1));
    asm("v_cvt_i32_f64 %0, %1" : "=v"(jy) : "v"(f2));
    const bool in = (int)((uint32_t)jx < (uint32_t)g.npix) & (int)((uint32_t)jy < (uint32_t)g.npix);
    ix = in ? jx : -1;
    iy = in ? jy : -1;
}

// What a lane of k_level3 holds for its ray column.
struct L3Lane {
    int64_t i;                 // ray column
    int32_t i32;
    bool in_col;               // the column lies inside the ray grid
    bool corner_col;           // ... in the first or last level-1 column
    bool wave_corner;          // some lane of the wave is (wave-uniform); rays of
                               // the four corner cells are left to k_level3_corner
    double t1, hr;             // theta_1, its offset from the level-2 column
    double c1, s1;             // beta_1 + S/2 without lens terms; kappa_* hr
    uint32_t coff;             // byte offset of the lane's level-2 point in a row
};

// Rows k0 <= k < k1 of a wave (k0, k1, jw wave-uniform): the level-2 series
// (coefficients reloaded when the level-2 row changes, a wave-uniform test),
// the corner cells' sheet, beta + S/2 and the pixel.  The series
// A(h) = sum_k C_k h^k, h = hr + i hi, is re-expanded at each reload about the
// lane's own column offset hr (a Taylor shift by synthetic division:
// A = sum_j D_j (i hi)^j), so that each row evaluates a polynomial in its
// real hi.
// FULL: every ray of these rows lies in [ray_first, ray_last).  BIN: pixels
// into pxs/pys (-1 for rays not binned); otherwise the per-ray outputs.
template <bool BIN, bool FULL>
__device__ __forceinline__ void level3_rows(
    const DevGeom &g, const RowInfo *__restrict__ rows, const double *__restrict__ coef,
    int32_t cy0, int64_t nxq, const L3Lane &ln, int32_t jw, int k0, int k1, int64_t ray_first,
    int64_t ray_last, const double *n1s, const double *n2s, double *a1o, double *a2o,
    int64_t *pixo, int32_t *pxs, int32_t *pys)
{
    constexpr int R = kL3RowsPerWave;
    const int32_t ny1 = (int32_t)g.ny - 1;
    double2 C[5] = {};
    int32_t cgy = -1;                                     // level-2 row held in C
#pragma unroll
    for (int k = 0; k < R; ++k) {
        pxs[k] = -1;
        pys[k] = -1;
        if (k < k0 || k >= k1) continue;                  // wave-uniform
        const RowInfo &rk = rows[min(jw + k, ny1)];
        const int32_t gy = rk.gy;
        if (gy != cgy) {                                  // wave-uniform: next level-2 row
            const double2 *cp = (const double2 *)((const char *)(coef + (int64_t)(gy - cy0 * g.q) *
                                                                          nxq * 10) + ln.coff);
#pragma unroll
            for (int e = 0; e < 5; ++e) C[e] = cp[e];
            // D_j = sum_{k >= j} binom(k, j) C_k hr^(k-j), in place
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int o = 3; o >= j; --o) {
                    C[o].x = fma(ln.hr, C[o + 1].x, C[o].x);
                    C[o].y = fma(ln.hr, C[o + 1].y, C[o].y);
                }
            cgy = gy;
        }
        const double hi = rk.hi;
        // A = sum_j D_j (i hi)^j with i^j = 1, i, -1, -i, 1: Horner in hi,
        // one fused multiply-add per component and step; conj(A) is the far
        // deflection
        const double Ar =
            fma(fma(fma(fma(C[4].x, hi, C[3].y), hi, -C[2].x), hi, -C[1].y), hi, C[0].x);
        const double Ai =
            fma(fma(fma(fma(C[4].y, hi, -C[3].x), hi, -C[2].y), hi, C[1].x), hi, C[0].y);
        // beta + S/2 = (c1, c2) - nearby lenses - conj(A)
        const double xs1 = (ln.c1 - n1s[k]) - Ar;
        const double xs2 = (rk.c2 - n2s[k]) + Ai;
        bool valid;
        if constexpr (FULL) {
            valid = ln.in_col;
        } else {
            // columns of row k inside [ray_first, ray_last), as a lane window
            const int64_t lo = ray_first - rk.base, hi_ = ray_last - rk.base;
            const int32_t wlo = (int32_t)(lo < 0 ? 0 : (lo > g.nx ? g.nx : lo));
            const int32_t whi = (int32_t)(hi_ < 0 ? 0 : (hi_ > g.nx ? g.nx : hi_));
            // (lanes past a narrow tile's end hold columns of the next tile)
            valid = (int)ln.in_col & (int)(ln.i32 >= wlo) & (int)(ln.i32 < whi);
        }
        // rays of the rectangle's four corner cells are k_level3_corner's
        if (ln.wave_corner && (rk.cy == 0 || rk.cy == g.n1y - 1)) valid = valid && !ln.corner_col;
        int32_t px, py;
        pixel_pair(g, xs1, xs2, px, py);
        pxs[k] = valid ? px : -1;
        pys[k] = valid ? py : -1;
        if (!BIN && valid) {
            const double s2 = g.sheet ? g.kappa_star * hi : 0.0;
            const double a1 = fma(g.kpg, ln.t1, n1s[k]) + (Ar - ln.s1);
            const double a2 = fma(g.kmg, rk.t2, n2s[k]) - (Ai + s2);
            const int64_t o = rk.base + ln.i - ray_first;
            if (a1o) a1o[o] = a1;
            if (a2o) a2o[o] = a2;
            if (pixo) pixo[o] = px < 0 ? -1 : (int64_t)py * g.npix + px;
        }
    }
}

// What a level-3 launch needs of one map (a kernel argument for a single
// map; a device table entry for a batch).
struct L3Map {
    DevGeom g;
    const double2 *lxy;             // sorted lenses (x, y)
    const double *lm;               // masses (null: unit)
    const int32_t *cell_start;
    const RowInfo *rows;            // row table
    const ColInfo *cols;            // column table
    const double *coef;             // level-2 coefficients from level-1 row cy0
    const TileSpan *tcol, *trow;    // the plan's column and row tiles
    int32_t cy0;
    int32_t ntx;                    // column tiles
    int64_t jr0, jr1;               // ray rows of the launch
    int64_t ray_first, ray_last;    // ray indices (per-ray outputs)
    double *a1o, *a2o;              // per-ray outputs, indexed r - ray_first, or
    int64_t *pixo;                  //   ... null
    uint32_t *counts;               // BIN: the map
    unsigned long long *landed;     // BIN: landed-ray counters
    // batches (whole maps): tiles and the corner cells' blocks of rays
    int32_t nty;                    // row tiles
    int32_t ncorner;                // corner cells with rays (<= 4)
    int64_t tiles;                  // nty * (ntx padded to a multiple of the XCDs)
    int64_t corner[4][4];           // their ray columns [0], [1) and rows [2], [3)
    int64_t corner_items[5];        // prefix of the corners' blocks of kThreads rays
};

// One tile of rays: columns tcol[tx] (one per lane) by rows trow[ty]
// (kL3RowsPerWave per wave), restricted to rows [jr0, jr1).  Every ray: the
// near lenses exactly, Horner of its level-2 point's C_0..C_4, the macro
// term, beta and the pixel; BIN: binned through an LDS histogram over the
// tile's landed-pixel box (flushed with one global atomic per non-empty bin),
// or, for a box larger than the histogram, global adds by runs of equal
// pixels down a lane's rows.  Called by every thread of the workgroup.
template <bool UNIT, bool BIN>
__device__ __forceinline__ void level3_tile(const L3Map &m, int32_t tx, int32_t ty, L3Lds *lds)
{
    const DevGeom &g = m.g;
    const int tid = threadIdx.x;
    const int lane = tid % kWave;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    constexpr int R = kL3RowsPerWave;
    const TileSpan tc = m.tcol[tx], tr = m.trow[ty];
    const int32_t ny1 = (int32_t)g.ny - 1;                          // ny < 2^31
    const int32_t jw = tr.a + wave * R;                             // the wave's first row
    if (BIN && tid == 0) {                    // one tile per workgroup: set up its LDS
        lds->bmin[0] = lds->bmin[1] = UINT32_MAX;
        lds->bmax[0] = lds->bmax[1] = -1;
        lds->landed = 0u;
    }
    __syncthreads();
    const int32_t i32 = tc.a + lane;
    const int64_t i = i32;
    const bool in_col = i32 < tc.b;
    const int64_t nxq = (int64_t)g.n1x * g.q;
    // the lane's column (lanes past the tile's end take its first column and
    // bin nothing); what the rows need of it is read after the lens pass
    const int32_t ic = in_col ? i32 : tc.a;
    const ColInfo *col = &m.cols[ic];
    const int32_t cx = col->cx;
    const double t1 = ray_x32(g, ic);
    const int32_t xl = cx > 0 ? cx - 1 : 0, xh = cx < g.n1x - 1 ? cx + 1 : g.n1x - 1;

    // the wave's rows jw + k, k < kt, lie in the tile; rows k0 <= k < k1 also
    // lie in [jr0, jr1), the others bin nothing
    const int kt = max(0, min(R, tr.b - jw));
    const int k0 = (int)max<int64_t>(0, m.jr0 - jw);
    const int k1 = (int)min<int64_t>(kt, m.jr1 - jw);
    auto row = [&](int k) -> const RowInfo & { return m.rows[min(jw + k, ny1)]; };

    // nearby lenses, exactly.  A lane's rays are R consecutive rows of one
    // column; they nearly always share their level-1 cell row (always where
    // row tiles follow the cell rows), so one pass over the lenses serves them
    // all, the R rows sharing each reciprocal; otherwise each ray takes its
    // own pass.  Which of the two a ray takes, and its partners in the first,
    // depend only on the plan's tiles, not on the call.
    double n1s[R], n2s[R], t2s[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        n1s[k] = 0.0;
        n2s[k] = 0.0;
        t2s[k] = row(k).t2;              // wave-uniform: kept in scalar registers
    }
    if (k1 > k0) {                                        // wave-uniform rows
        // level-1 columns of the wave's first and last ray (the tile's first
        // and last columns: the level-1 column grows with the ray column)
        const int32_t cxa = m.cols[tc.a].cx;
        const int32_t cxb = m.cols[tc.b - 1].cx;
        const int32_t cl = cxa > 0 ? cxa - 1 : 0, ch = cxb < g.n1x - 1 ? cxb + 1 : g.n1x - 1;
        const bool straddle = cxa != cxb;
        const int32_t cy0r = row(0).cy;
        if (row(kt - 1).cy == cy0r) {                     // rows sorted: all share cy0r
            if (straddle)
                near_pass<UNIT, R, true>(g, m.lxy, m.lm, m.cell_start, cy0r, cl, ch, true, xl, xh,
                                         t1, t2s, n1s, n2s);
            else
                near_pass<UNIT, R, false>(g, m.lxy, m.lm, m.cell_start, cy0r, cl, ch, false, xl,
                                          xh, t1, t2s, n1s, n2s);
        } else {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                if (k < k0 || k >= k1) continue;
                near_pass<UNIT, 1, true>(g, m.lxy, m.lm, m.cell_start, row(k).cy, cl, ch,
                                         straddle, xl, xh, t1, &t2s[k], &n1s[k], &n2s[k]);
            }
        }
    }

    // per-row evaluation; rows whose rays all lie in [ray_first, ray_last)
    // need no per-ray window test
    const bool full = k1 > k0 && row(k0).base >= m.ray_first &&
                      row(k1 - 1).base + g.nx <= m.ray_last;
    const bool corner_col = in_col && (cx == 0 || cx == g.n1x - 1);
    const bool wave_corner = g.sheet && __ballot(corner_col) != 0;     // wave-uniform
    const double hr = col->hr;
    double c1, s1;
    column_terms(g, t1, hr, c1, s1);
    const L3Lane ln{i, i32, in_col, corner_col, wave_corner, t1, hr, c1, s1, col->coff};
    int32_t pxs[R], pys[R];
    if (full)
        level3_rows<BIN, true>(g, m.rows, m.coef, m.cy0, nxq, ln, jw, k0, k1, m.ray_first,
                               m.ray_last, n1s, n2s, m.a1o, m.a2o, m.pixo, pxs, pys);
    else
        level3_rows<BIN, false>(g, m.rows, m.coef, m.cy0, nxq, ln, jw, k0, k1, m.ray_first,
                                m.ray_last, n1s, n2s, m.a1o, m.a2o, m.pixo, pxs, pys);
    if (!BIN) return;

    // the block's box of landed pixels and its landed rays: per row of 16
    // lanes by cross-lane reductions, then across the rows and waves by LDS
    // atomics.  A ray not binned has pixel -1, the largest unsigned value
    // (never a minimum) and the smallest signed one (never a maximum)
    uint32_t ux0 = UINT32_MAX, uy0 = UINT32_MAX;
    int bx1 = -1, by1 = -1, wl = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        ux0 = min(ux0, (uint32_t)pxs[k]); bx1 = max(bx1, pxs[k]);
        uy0 = min(uy0, (uint32_t)pys[k]); by1 = max(by1, pys[k]);
        wl += __popcll(__ballot(pxs[k] >= 0));              // landed rays of the wave's row
    }
    ux0 = row_min_u(ux0);
    uy0 = row_min_u(uy0);
    bx1 = row_max(bx1);
    by1 = row_max(by1);
    if (lane % 16 == 15) {
        atomicMin(&lds->bmin[0], ux0);
        atomicMin(&lds->bmin[1], uy0);
        atomicMax(&lds->bmax[0], bx1);
        atomicMax(&lds->bmax[1], by1);
    }
    if (lane == 0 && wl) atomicAdd(&lds->landed, (uint32_t)wl);
    __syncthreads();
    // every lane reads the same words: uniform values, in scalar registers
    const int bx0 = __builtin_amdgcn_readfirstlane((int)min(lds->bmin[0], (uint32_t)INT_MAX));
    const int by0 = __builtin_amdgcn_readfirstlane((int)min(lds->bmin[1], (uint32_t)INT_MAX));
    bx1 = __builtin_amdgcn_readfirstlane(lds->bmax[0]);
    by1 = __builtin_amdgcn_readfirstlane(lds->bmax[1]);
    const int nblock = __builtin_amdgcn_readfirstlane((int)lds->landed);
    if (tid == 0 && nblock) landed_add(m.landed, (unsigned long long)nblock);
    if (bx1 < 0) return;                                   // nothing landed (block-uniform)
    // histogram rows of pitch 2^sh >= the box's width
    const int sh = 32 - __clz(bx1 - bx0);
    const int64_t area = (int64_t)(by1 - by0 + 1) << sh;
    uint32_t *counts = m.counts;
    if (area > kHistCap) {
        // block-uniform fallback (rays scattered, as near a lens): global
        // adds by runs of equal pixels down a lane's rows
        int32_t cur = -1;
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int32_t pix = pxs[k] < 0 ? -1 : pys[k] * g.npix + pxs[k];
            if (pix == cur) {
                ++run;
                continue;
            }
            if (cur >= 0) atomicAdd(&counts[cur], run);
            cur = pix;
            run = 1;
        }
        if (cur >= 0) atomicAdd(&counts[cur], run);
        return;
    }
    const int nbin = (int)area;
    for (int b = tid; b < nbin; b += kThreads) lds->hist[b] = 0u;
    // byte offsets of a lane's bins; a ray not binned (pixel -1 in both
    // coordinates) gives a negative offset, which the unsigned minimum turns
    // into the spare bin's
    uint32_t lb[R];
    const uint32_t spare = (uint32_t)kHistCap * 4u;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const uint32_t xb = (uint32_t)(pxs[k] - bx0) * 4u;
        lb[k] = min(((uint32_t)(pys[k] - by0) << (sh + 2)) + xb, spare);
    }
    __syncthreads();
    // LDS adds by runs: a lane's rays are consecutive rows of one column and
    // mostly land in one pixel, so each run of equal bins is added once, at
    // its last row
    {
        char *h = (char *)lds->hist;
        int first = 0;                                     // the current run's first row
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (k == R - 1 || lb[k] != lb[k + 1]) {
                atomicAdd((uint32_t *)(h + lb[k]), (uint32_t)(k + 1 - first));
                first = k + 1;
            }
        }
    }
    __syncthreads();
    // flush: bin b is (row b >> sh, column b & (2^sh - 1)) of the box
    const int colmask = (1 << sh) - 1;
    for (int b = tid; b < nbin; b += kThreads) {
        const uint32_t v = lds->hist[b];
        if (v) atomicAdd(&counts[(by0 + (b >> sh)) * g.npix + bx0 + (b & colmask)], v);
    }
}

// One map: tile (tx, ty0 + blockIdx.x / ntx_pad) with tx = blockIdx.x mod
// ntx_pad.  ntx_pad is a multiple of the 8 XCDs, which take consecutive
// workgroups in turn, so a column tile runs on the same XCD in every tile row
// and finds its level-2 coefficients and lenses in that XCD's L2.
template <bool UNIT, bool BIN>
__global__ __launch_bounds__(kThreads, 5) void k_level3(L3Map m, int32_t ty0, int32_t ntx_pad)
{
    __shared__ L3Lds lds;
    const int32_t tx = (int32_t)(blockIdx.x % (uint32_t)ntx_pad);
    if (tx >= m.ntx) return;                               // padding (block-uniform)
    level3_tile<UNIT, BIN>(m, tx, ty0 + (int32_t)(blockIdx.x / (uint32_t)ntx_pad), &lds);
}

// Ray idx of one of the rectangle's four corner cells (ray columns [i0, i1),
// rows [j0, j1)), which k_level3 leaves out: the sheet's series does not
// converge over a corner cell, so these rays take its closed form.  Nearby
// lenses one by one (near_term), the level-2 series, the sheet's closed
// form, beta, the pixel.  BIN: a global add into counts and the landed
// counters; otherwise the per-ray outputs of rays in [ray_first, ray_last).
// Called by every lane of a wave.
template <bool UNIT, bool BIN>
__device__ __forceinline__ void level3_corner_ray(const L3Map &m, int64_t i0, int64_t i1,
                                                  int64_t j0, int64_t j1, int64_t idx)
{
    const DevGeom &g = m.g;
    const int64_t ncol = i1 - i0;
    const bool inside = idx < ncol * (j1 - j0);
    const int64_t i = inside ? i0 + idx % ncol : i0;
    const RowInfo &rk = m.rows[inside ? j0 + idx / ncol : j0];
    const int64_t r = rk.base + i;
    const bool valid = inside && r >= m.ray_first && r < m.ray_last;
    const int64_t nxq = (int64_t)g.n1x * g.q;
    const int64_t gx = floor_div((2 * i + 1) * nxq, 2 * g.nx);
    const int32_t cx = (int32_t)(gx / g.q), cy = rk.cy;
    const double t1 = ray_x(g, i);
    const double hr = t1 - level2_x(g, gx);
    const double s1 = g.kappa_star * hr;
    const double mac1 = g.kpg * t1;
    const double c1 = ((t1 - mac1) + s1) + g.half_side;
    double n1 = 0.0, n2 = 0.0;
    const int32_t xl = cx > 0 ? cx - 1 : 0, xh = cx < g.n1x - 1 ? cx + 1 : g.n1x - 1;
    const int32_t yl = cy > 0 ? cy - 1 : 0, yh = cy < g.n1y - 1 ? cy + 1 : g.n1y - 1;
    for (int32_t row = yl; row <= yh; ++row) {
        const int32_t pe = m.cell_start[row * g.n1x + xh + 1];
        for (int32_t q_ = m.cell_start[row * g.n1x + xl]; q_ < pe; ++q_) {
            const double2 z = m.lxy[q_];
            const double d1 = t1 - z.x;
            near_term(d1, fma(d1, d1, kNearTiny), rk.t2, z.y, UNIT ? 1.0 : m.lm[q_], n1, n2);
        }
    }
    const double2 *cp =
        (const double2 *)(m.coef + ((int64_t)(rk.gy - m.cy0 * g.q) * nxq + gx) * 10);
    double Ar = cp[4].x, Ai = cp[4].y;
#pragma unroll
    for (int o = 3; o >= 0; --o) {
        const double t = fma(Ar, hr, fma(-Ai, rk.hi, cp[o].x));
        Ai = fma(Ar, rk.hi, fma(Ai, hr, cp[o].y));
        Ar = t;
    }
    const D2 d = corner_sheet(g, t1, rk.t2, hr, rk.hi);
    Ar += d.x;
    Ai += d.y;
    const double xs1 = (c1 - n1) - Ar;
    const double xs2 = (rk.c2 - n2) + Ai;
    int32_t px, py;
    pixel_pair(g, xs1, xs2, px, py);
    if (BIN) {
        const bool bin = valid && px >= 0;
        if (bin) atomicAdd(&m.counts[py * g.npix + px], 1u);
        const uint64_t got = __ballot(bin);
        if (__lane_id() == 0 && got) landed_add(m.landed, (unsigned long long)__popcll(got));
    } else if (valid) {
        const double s2 = g.kappa_star * rk.hi;
        const int64_t o = r - m.ray_first;
        if (m.a1o) m.a1o[o] = fma(g.kpg, t1, n1) + (Ar - s1);
        if (m.a2o) m.a2o[o] = fma(g.kmg, rk.t2, n2) - (Ai + s2);
        if (m.pixo) m.pixo[o] = px < 0 ? -1 : (int64_t)py * g.npix + px;
    }
}

// One corner cell's rays of a map, one per lane.
template <bool UNIT, bool BIN>
__global__ __launch_bounds__(kThreads) void k_level3_corner(L3Map m, int64_t i0, int64_t i1,
                                                            int64_t j0, int64_t j1)
{
    level3_corner_ray<UNIT, BIN>(m, i0, i1, j0, j1,
                                 (int64_t)blockIdx.x * kThreads + threadIdx.x);
}

// A batch's level 3 as one launch over every map's tiles.  The maps'
// arguments sit in a table in device memory that does not change during the
// launch.  Read through the constant address space, its fields come in scalar
// loads that the compiler may repeat where it needs them, as it does for
// kernel arguments, so the tile routine stays within five waves' registers;
// read through a plain pointer it spilled.
typedef const __attribute__((address_space(4))) L3Map ConstL3Map;
typedef const __attribute__((address_space(4))) int64_t ConstI64;

// The tiles of n maps laid end to end (start[k] = map k's first tile,
// start[n] = all tiles; a map's column tiles padded to a multiple of the
// XCDs, so every start[k] is one too).  Workgroup (x, y) takes tile
// y gridDim.x + x, gridDim.x a multiple of the XCDs: a column tile always runs
// on the same XCD, and the dispatcher hands the tiles out in order, longest
// map first.  (A grid-stride loop over the tiles made the compiler spill.)
template <bool UNIT>
__global__ __launch_bounds__(kThreads, 5) void k_level3_maps(const L3Map *maps_in,
                                                             const int64_t *start_in, int32_t n)
{
    __shared__ L3Lds lds;
    ConstL3Map *maps = (ConstL3Map *)maps_in;
    ConstI64 *start = (ConstI64 *)start_in;
    const int64_t t = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (t >= start[n]) return;                              // the last grid row's tail
    int32_t lo = 0, hi = n;                                 // start[lo] <= t < start[hi]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (start[mid] <= t) lo = mid;
        else hi = mid;
    }
    const L3Map &m = *(const L3Map *)&maps[lo];
    const int64_t local = t - start[lo];
    const int32_t ntx_pad = (m.ntx + kXcds - 1) / kXcds * kXcds;
    const int32_t tx = (int32_t)(local % ntx_pad);
    if (tx < m.ntx)                                         // padding (block-uniform)
        level3_tile<UNIT, true>(m, tx, (int32_t)(local / ntx_pad), &lds);
}

// The same maps' corner-cell rays: block b takes kThreads rays of one corner
// cell (the maps' corner blocks laid end to end, cstart like start).
template <bool UNIT>
__global__ __launch_bounds__(kThreads) void k_level3_maps_corners(const L3Map *maps_in,
                                                                  const int64_t *cstart_in,
                                                                  int32_t n)
{
    ConstL3Map *maps = (ConstL3Map *)maps_in;
    ConstI64 *cstart = (ConstI64 *)cstart_in;
    const int64_t bt = blockIdx.x;
    int32_t k = 0;
    while (k + 1 < n && cstart[k + 1] <= bt) ++k;
    const L3Map &m = *(const L3Map *)&maps[k];
    const int64_t ci = bt - cstart[k];
    int c = 0;
    while (c + 1 < m.ncorner && m.corner_items[c + 1] <= ci) ++c;
    level3_corner_ray<UNIT, true>(m, m.corner[c][0], m.corner[c][1], m.corner[c][2],
                                  m.corner[c][3],
                                  (ci - m.corner_items[c]) * kThreads + threadIdx.x);
}

// first ray row j with level2_row(j) >= G (level2_row is non-decreasing)
int64_t first_row_at(const DevGeom &g, int64_t G)
{
    int64_t lo = 0, hi = g.ny;
    const int64_t M = (int64_t)g.n1y * g.q;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (((2 * mid + 1) * M) / (2 * g.ny) >= G) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

int64_t level2_row_host(const DevGeom &g, int64_t j)
{
    return ((2 * j + 1) * (int64_t)g.n1y * g.q) / (2 * g.ny);
}

}  // namespace

// Expansion order of the per-cell local expansion (0: sum at every point as
// in the paper).  The expansion about a cell centre converges over the cell
// with ratio rho = (half diagonal)/((R + 1/2) * shorter side); the truncation
// of c_4 is about C(P,4) rho^(P-4)/(1-rho)^5, kept below 1e-14.
int level2_order(const irs_plan_s *p)
{
    if (p->params.flags & IRS_LEVEL2_PAPER) return 0;
    const DevGeom &g = p->dg;
    const double rho = 0.5 * std::sqrt(g.w1 * g.w1 + g.h1 * g.h1) /
                       ((kRing + 0.5) * std::min(g.w1, g.h1));
    for (int P : {32, 48}) {
        double c4 = (double)P * (P - 1) * (P - 2) * (P - 3) / 24.0;
        if (c4 * std::pow(rho, P - 4) / std::pow(1.0 - rho, 5) < 1e-14) return P;
    }
    return 0;
}

namespace {

int64_t level2_row_bytes(const irs_plan_s *p)
{
    return (int64_t)p->dg.n1x * p->dg.q * p->dg.q * 10 * (int64_t)sizeof(double);
}

// level-1 rows per band: as many as fit in the plan's coefficient budget
int64_t band_rows(const irs_plan_s *p)
{
    return std::min<int64_t>(p->dg.n1y, std::max<int64_t>(1, p->coef_budget / level2_row_bytes(p)));
}

// partial-expansion buffer for `rows` level-1 rows
irs_status ensure_part(irs_plan_s *p, int64_t rows)
{
    const int P = level2_order(p);
    if (P <= 0) return IRS_OK;
    const size_t need = (size_t)rows * p->dg.n1x * level2_chunks(p) * P * 2 * sizeof(double);
    if (p->part_bytes < need) {
        irs_status st = alloc_allowed(p, "the level-2 cell expansions");
        if (st != IRS_OK) return st;
        dev_free(p->d_part);
        p->d_part = nullptr;
        p->part_bytes = 0;
        if (dev_alloc(&p->d_part, need) != hipSuccess) {
            (void)hipGetLastError();
            set_error("cannot allocate the level-2 partial expansions");
            return IRS_E_NOMEM;
        }
        p->part_bytes = need;
    }
    return IRS_OK;
}

// coefficient and partial-expansion buffers for bands of `rows` level-1 rows
irs_status ensure_bands(irs_plan_s *p, int64_t rows)
{
    if (p->coef_rows_cap < rows) {
        irs_status st = alloc_allowed(p, "the level-2 coefficient band");
        if (st != IRS_OK) return st;
        dev_free(p->d_coef);
        p->d_coef = nullptr;
        p->coef_rows_cap = 0;
        p->coef_c0 = -1;
        p->coef_c1 = -2;
        if (dev_alloc(&p->d_coef, (size_t)(rows * level2_row_bytes(p))) != hipSuccess) {
            (void)hipGetLastError();
            set_error("cannot allocate the level-2 coefficient band");
            return IRS_E_NOMEM;
        }
        p->coef_rows_cap = rows;
    }
    return ensure_part(p, p->coef_rows_cap);
}

}  // namespace

int super_order(const irs_plan_s *p)
{
    if (level2_order(p) == 0) return 0;
    const DevGeom &g = p->dg;
    // the super block's half-diagonal over the distance to the nearest
    // excluded lens: independent of the super-cell side
    const double rho = 0.5 * std::sqrt(g.w1 * g.w1 + g.h1 * g.h1) /
                       ((kSuperR + 0.5) * std::min(g.w1, g.h1));
    for (int P : {32, 40, 48}) {
        double c4 = (double)P * (P - 1) * (P - 2) * (P - 3) / 24.0;
        if (c4 * std::pow(rho, P - 4) / std::pow(1.0 - rho, 5) < 1e-14) return P;
    }
    return 0;
}

int32_t level2_chunks(const irs_plan_s *p)
{
    if (super_order(p) > 0) return 1;
    return p->n_lens > 0 ? (int32_t)((p->n_lens + kChunkLens - 1) / kChunkLens) : 1;
}

void level2_reset(irs_plan_s *p)
{
    std::fill(p->super_ok.begin(), p->super_ok.end(), 0);
    std::fill(p->mid_ok.begin(), p->mid_ok.end(), 0);
    p->coef_c0 = -1;                 // no band of coefficients resident either
    p->coef_c1 = -2;
}

// Super-cell side K_S and mid-cell side K_M (cells; K_M = 0: no mid level),
// once per plan.  Work in series terms, with nu lenses per cell and B(K) =
// min(N_*, nu (2 R_S + 1)^2 K^2) the lenses of a 5 x 5 block of K x K cells:
//   super expansions  N_* (cells / K_S^2) PS
//   mid expansions    (cells / K_M^2) (B(K_S) PS + PS^2)
//   cell expansions   cells (B(K_M or K_S) P + PS P)
// over K_S in {4, .., 32} and K_M in {0, 4, 8} with K_S a multiple of
// kCellsPerBlock K_M (a workgroup's kCellsPerBlock children must share one
// parent); the accuracy of every series is that of the order rule whatever
// the sides.
void choose_sides(irs_plan_s *p)
{
    if (p->super_k > 0) return;
    const DevGeom &g = p->dg;
    const double cells = (double)g.n1x * (double)g.n1y, nl = (double)p->n_lens;
    const double nu = cells > 0.0 ? nl / cells : 0.0;
    const double PS = std::max(1, super_order(p)), P = std::max(1, level2_order(p));
    auto block = [&](int32_t K) {
        const double b = (double)(2 * kSuperR + 1) * K;
        return std::min(nl, nu * b * b);
    };
    auto count = [&](int32_t K) { return std::ceil(g.n1x / (double)K) * std::ceil(g.n1y / (double)K); };
    int32_t bs = 8, bm = 0;
    double best = -1.0;
    for (int32_t KS : {4, 8, 16, 32})
        for (int32_t KM : {0, 4, 8}) {
            if (KM != 0 && KS % (kCellsPerBlock * KM) != 0) continue;
            double cost = nl * count(KS) * PS + cells * PS * P;
            if (KM == 0) cost += cells * block(KS) * P;
            else cost += count(KM) * (block(KS) * PS + PS * PS) + cells * block(KM) * P;
            if (best < 0.0 || cost < best) {
                best = cost;
                bs = KS;
                bm = KM;
            }
        }
    p->super_k = bs;
    p->mid_k = bm;
}

int32_t super_side(irs_plan_s *p)
{
    choose_sides(p);
    return p->super_k;
}

int32_t mid_side(irs_plan_s *p)
{
    choose_sides(p);
    return p->mid_k;
}

namespace {

int32_t super_nx(irs_plan_s *p) { const int32_t k = super_side(p); return (p->dg.n1x + k - 1) / k; }
int32_t super_ny(irs_plan_s *p) { const int32_t k = super_side(p); return (p->dg.n1y + k - 1) / k; }
int32_t lens_chunks(const irs_plan_s *p)
{
    return p->n_lens > 0 ? (int32_t)((p->n_lens + kChunkLens - 1) / kChunkLens) : 1;
}

irs_status ensure_super_buffers(irs_plan_s *p, int64_t rows)
{
    const int PS = super_order(p);
    const int32_t nSx = super_nx(p), nSy = super_ny(p);
    if (!p->d_super) {
        irs_status st = alloc_allowed(p, "the super-cell expansions");
        if (st != IRS_OK) return st;
        if (dev_alloc(&p->d_super, sizeof(double) * (size_t)nSy * nSx * PS * 2) != hipSuccess) {
            (void)hipGetLastError();
            p->d_super = nullptr;
            set_error("cannot allocate the super-cell expansions");
            return IRS_E_NOMEM;
        }
        p->super_ok.assign((size_t)nSy, 0);
    }
    const size_t need = sizeof(double) * (size_t)rows * nSx * lens_chunks(p) * PS * 2;
    if (p->super_part_bytes < need) {
        irs_status st = alloc_allowed(p, "the super-cell partial expansions");
        if (st != IRS_OK) return st;
        dev_free(p->d_super_part);
        p->d_super_part = nullptr;
        p->super_part_bytes = 0;
        if (dev_alloc(&p->d_super_part, need) != hipSuccess) {
            (void)hipGetLastError();
            set_error("cannot allocate the super-cell partial expansions");
            return IRS_E_NOMEM;
        }
        p->super_part_bytes = need;
    }
    return IRS_OK;
}

// lenses of the cell block [xa, xb) x [ya, yb) (clipped), from the host copy
int64_t lenses_in(const irs_plan_s *p, int64_t xa, int64_t xb, int64_t ya, int64_t yb)
{
    const DevGeom &g = p->dg;
    xa = std::max<int64_t>(0, xa);
    xb = std::min<int64_t>(g.n1x, xb);
    ya = std::max<int64_t>(0, ya);
    yb = std::min<int64_t>(g.n1y, yb);
    if (xa >= xb || ya >= yb) return 0;
    const std::vector<int32_t> &hc = p->h_cell_start;
    int64_t n = 0;
    for (int64_t row = ya; row < yb; ++row) n += hc[row * g.n1x + xb] - hc[row * g.n1x + xa];
    return n;
}

// whether every workgroup of the level-2 points kernel (four cells of a row)
// finds its cells' ring lenses, a block of 7 x 10 cells, within kRingCap;
// computed once per plan from the host copy of the cell table
bool ring_fits(irs_plan_s *p)
{
    if (p->ring_fit < 0) {
        const DevGeom &g = p->dg;
        bool ok = true;
        for (int64_t cy = 0; cy < g.n1y && ok; ++cy)
            for (int64_t cx0 = 0; cx0 < g.n1x && ok; cx0 += kCellsPerBlock)
                ok = lenses_in(p, cx0 - kRing, cx0 + kCellsPerBlock + kRing, cy - kRing,
                               cy + kRing + 1) <= kRingCap;
        p->ring_fit = ok ? 1 : 0;
    }
    return p->ring_fit == 1;
}

// super rows [Ya, Yb] that are not cached, in runs of consecutive rows
irs_status ensure_super_rows(irs_plan_s *p, int64_t Ya, int64_t Yb, double *flops)
{
    const DevGeom &g = p->dg;
    const int PS = super_order(p);
    const int32_t ks = super_side(p);
    const int32_t nSx = super_nx(p);
    const int32_t nSxb = (nSx + kCellsPerBlock - 1) / kCellsPerBlock;
    const int32_t nchunk = lens_chunks(p);
    const int32_t nl = (int32_t)p->n_lens;
    irs_status st = ensure_super_buffers(p, 1);
    if (st != IRS_OK) return st;
    for (int64_t y0 = Ya; y0 <= Yb;) {
        if (p->super_ok[y0]) { ++y0; continue; }
        int64_t y1 = y0;
        while (y1 + 1 <= Yb && !p->super_ok[y1 + 1]) ++y1;
        if ((st = ensure_super_buffers(p, y1 - y0 + 1)) != IRS_OK) return st;
        const unsigned nb = (unsigned)((y1 - y0 + 1) * nSxb * nchunk);
#define IRS_SE(U, PP)                                                                          \
    hipLaunchKernelGGL((k_super_expand<U, PP>), dim3(nb), dim3(kThreads), 0, p->stream, g,      \
                       p->d_x, p->d_y, p->d_m, p->d_cxy, nl, (int32_t)y0, nSx, nSxb, nchunk,  \
                       kChunkLens, ks, p->d_super_part)
        if (p->unit_mass) {
            if (PS == 32) IRS_SE(true, 32);
            else if (PS == 40) IRS_SE(true, 40);
            else IRS_SE(true, 48);
        } else {
            if (PS == 32) IRS_SE(false, 32);
            else if (PS == 40) IRS_SE(false, 40);
            else IRS_SE(false, 48);
        }
#undef IRS_SE
        const int64_t n_out = (y1 - y0 + 1) * nSx * PS * 2;
        hipLaunchKernelGGL(k_super_reduce, dim3((unsigned)((n_out + kThreads - 1) / kThreads)),
                           dim3(kThreads), 0, p->stream, p->d_super_part, n_out, nchunk, PS,
                           p->d_super + y0 * nSx * PS * 2);
        IRS_HIP(hipGetLastError());
        if (flops)
            for (int64_t Y = y0; Y <= y1; ++Y)
                for (int32_t X = 0; X < nSx; ++X) {
                    const int64_t inside = lenses_in(p, (X - kSuperR) * ks, (X + kSuperR + 1) * ks,
                                                     (Y - kSuperR) * ks, (Y + kSuperR + 1) * ks);
                    *flops += (double)(p->n_lens - inside) * (10.0 + 8.0 * PS);
                }
        for (int64_t Y = y0; Y <= y1; ++Y) p->super_ok[Y] = 1;
        y0 = y1 + 1;
    }
    return IRS_OK;
}

int32_t mid_nx(irs_plan_s *p) { const int32_t k = mid_side(p); return (p->dg.n1x + k - 1) / k; }
int32_t mid_ny(irs_plan_s *p) { const int32_t k = mid_side(p); return (p->dg.n1y + k - 1) / k; }

irs_status ensure_mid_buffers(irs_plan_s *p)
{
    if (p->d_mid) return IRS_OK;
    irs_status st = alloc_allowed(p, "the mid-cell expansions");
    if (st != IRS_OK) return st;
    const int PS = super_order(p);
    const int32_t nMx = mid_nx(p), nMy = mid_ny(p);
    if (dev_alloc(&p->d_mid, sizeof(double) * (size_t)nMy * nMx * PS * 2) != hipSuccess) {
        (void)hipGetLastError();
        p->d_mid = nullptr;
        set_error("cannot allocate the mid-cell expansions");
        return IRS_E_NOMEM;
    }
    p->mid_ok.assign((size_t)nMy, 0);
    return IRS_OK;
}

// mid rows [Ma, Mb] that are not cached, in runs of consecutive rows: each mid
// cell takes its super cell's expansion re-expanded about its centre plus the
// lenses of the super block outside its own 5 x 5 block of mid cells
irs_status ensure_mid_rows(irs_plan_s *p, int64_t Ma, int64_t Mb, double *flops)
{
    const DevGeom &g = p->dg;
    const int PS = super_order(p);
    const int32_t ks = super_side(p), km = mid_side(p);
    if (km <= 0 || ks % (kCellsPerBlock * km) != 0) {
        set_error("internal: mid cells must tile their super cells by workgroups");
        return IRS_E_INVALID;
    }
    irs_status st = ensure_mid_buffers(p);
    if (st != IRS_OK) return st;
    if ((st = ensure_super_rows(p, Ma * km / ks, Mb * km / ks, flops)) != IRS_OK) return st;
    const int32_t nSx = super_nx(p), nMx = mid_nx(p);
    const int32_t nxb = (nMx + kCellsPerBlock - 1) / kCellsPerBlock;
    for (int64_t m0 = Ma; m0 <= Mb;) {
        if (p->mid_ok[m0]) { ++m0; continue; }
        int64_t m1 = m0;
        while (m1 + 1 <= Mb && !p->mid_ok[m1 + 1]) ++m1;
        const unsigned nb = (unsigned)((m1 - m0 + 1) * nxb);
        double *dst = p->d_mid + m0 * nMx * PS * 2;
#define IRS_MID(U, PP)                                                                          \
    hipLaunchKernelGGL((k_level2_near<U, PP, PP>), dim3(nb), dim3(kThreads), 0, p->stream, g,    \
                       p->d_x, p->d_y, p->d_m, p->d_cxy, p->d_cell_start, p->d_super, nSx,     \
                       (int32_t)m0, nxb, ks, km, kSuperR, nMx, 0, dst)
        if (p->unit_mass) {
            if (PS == 32) IRS_MID(true, 32);
            else if (PS == 40) IRS_MID(true, 40);
            else IRS_MID(true, 48);
        } else {
            if (PS == 32) IRS_MID(false, 32);
            else if (PS == 40) IRS_MID(false, 40);
            else IRS_MID(false, 48);
        }
#undef IRS_MID
        IRS_HIP(hipGetLastError());
        if (flops)
            for (int64_t M = m0; M <= m1; ++M)
                for (int32_t X = 0; X < nMx; ++X) {
                    const int64_t SX = (int64_t)X * km / ks, SY = M * km / ks;
                    const int64_t ring =
                        lenses_in(p, (SX - kSuperR) * ks, (SX + kSuperR + 1) * ks,
                                  (SY - kSuperR) * ks, (SY + kSuperR + 1) * ks) -
                        lenses_in(p, ((int64_t)X - kSuperR) * km, ((int64_t)X + kSuperR + 1) * km,
                                  (M - kSuperR) * km, (M + kSuperR + 1) * km);
                    *flops += (double)ring * (10.0 + 8.0 * PS) + 8.0 * PS * PS;
                }
        for (int64_t M = m0; M <= m1; ++M) p->mid_ok[M] = 1;
        m0 = m1 + 1;
    }
    return IRS_OK;
}

}  // namespace

irs_status level2_prepare(irs_plan_s *p)
{
    level2_reset(p);
    if (super_order(p) <= 0) return IRS_OK;
    irs_status st = ensure_super_buffers(p, super_ny(p));
    if (st != IRS_OK || mid_side(p) == 0) return st;
    return ensure_mid_buffers(p);
}

irs_status launch_level2_expand(irs_plan_s *p, int64_t c0, int64_t c1, double *flops,
                                bool fold_sheet)
{
    const int P = level2_order(p);
    if (P <= 0) {
        set_error("the per-cell expansion is not used by this plan");
        return IRS_E_UNSUPPORTED;
    }
    irs_status st = ensure_part(p, c1 - c0 + 1);
    if (st != IRS_OK) return st;
    const DevGeom &g = p->dg;
    const int32_t nl = (int32_t)p->n_lens;
    const int32_t nxb = (g.n1x + kCellsPerBlock - 1) / kCellsPerBlock;
    const int PS = super_order(p);
    if (PS == 0) {
        // one level: every cell sums all its distant lenses, in lens chunks
        const int32_t nchunk = level2_chunks(p);
        const unsigned nb = (unsigned)((c1 - c0 + 1) * nxb * nchunk);
#define IRS_L2E(U, PP)                                                                    \
    hipLaunchKernelGGL((k_level2_expand<U, PP>), dim3(nb), dim3(kThreads), 0, p->stream, g, \
                       p->d_x, p->d_y, p->d_m, p->d_cxy, nl, (int32_t)c0, nxb, nchunk,   \
                       kChunkLens, p->d_part)
        if (p->unit_mass) {
            if (P == 32) IRS_L2E(true, 32);
            else IRS_L2E(true, 48);
        } else {
            if (P == 32) IRS_L2E(false, 32);
            else IRS_L2E(false, 48);
        }
#undef IRS_L2E
        IRS_HIP(hipGetLastError());
        if (flops)
            for (int64_t cy = c0; cy <= c1; ++cy)
                for (int64_t cx = 0; cx < g.n1x; ++cx)
                    *flops += (double)(p->n_lens - lenses_in(p, cx - kRing, cx + kRing + 1, cy - kRing,
                                                              cy + kRing + 1)) * (10.0 + 8.0 * P);
        return IRS_OK;
    }
    // the cells' parent level: mid cells if the plan has them, else super cells
    const int32_t km = mid_side(p);
    const int32_t ks = km > 0 ? km : super_side(p);
    if (km > 0) st = ensure_mid_rows(p, c0 / km, c1 / km, flops);
    else st = ensure_super_rows(p, c0 / ks, c1 / ks, flops);
    if (st != IRS_OK) return st;
    const double *parent = km > 0 ? p->d_mid : p->d_super;
    const int32_t nSx = km > 0 ? mid_nx(p) : super_nx(p);
    const unsigned nb = (unsigned)((c1 - c0 + 1) * nxb);
#define IRS_LN(U, PP, QS)                                                                         \
    hipLaunchKernelGGL((k_level2_near<U, PP, QS>), dim3(nb), dim3(kThreads), 0, p->stream, g,      \
                       p->d_x, p->d_y, p->d_m, p->d_cxy, p->d_cell_start, parent, nSx,          \
                       (int32_t)c0, nxb, ks, 1, kRing, g.n1x, fold_sheet ? 1 : 0, p->d_part)
    if (p->unit_mass) {
        if (P == 32) {
            if (PS == 32) IRS_LN(true, 32, 32);
            else if (PS == 40) IRS_LN(true, 32, 40);
            else IRS_LN(true, 32, 48);
        } else {
            if (PS == 32) IRS_LN(true, 48, 32);
            else if (PS == 40) IRS_LN(true, 48, 40);
            else IRS_LN(true, 48, 48);
        }
    } else {
        if (P == 32) {
            if (PS == 32) IRS_LN(false, 32, 32);
            else if (PS == 40) IRS_LN(false, 32, 40);
            else IRS_LN(false, 32, 48);
        } else {
            if (PS == 32) IRS_LN(false, 48, 32);
            else if (PS == 40) IRS_LN(false, 48, 40);
            else IRS_LN(false, 48, 48);
        }
    }
#undef IRS_LN
    IRS_HIP(hipGetLastError());
    if (flops)
        for (int64_t cy = c0; cy <= c1; ++cy) {
            const int64_t Y = cy / ks;
            for (int64_t cx = 0; cx < g.n1x; ++cx) {
                const int64_t X = cx / ks;
                const int64_t ring = lenses_in(p, (X - kSuperR) * ks, (X + kSuperR + 1) * ks,
                                               (Y - kSuperR) * ks, (Y + kSuperR + 1) * ks) -
                                     lenses_in(p, cx - kRing, cx + kRing + 1, cy - kRing, cy + kRing + 1);
                *flops += (double)ring * (10.0 + 8.0 * P) + 8.0 * PS * P;
            }
        }
    return IRS_OK;
}

// Tiles of one axis: where every level-1 cell spans at least `min_span` rays
// along it (and, with `weigh`, the lanes this leaves idle cost less than the
// extra lenses of tiles that straddle cells), tiles follow the cells (each
// cell's rays cut into tiles of at most `tile` rays from its first ray), so
// no wave straddles two cells; otherwise tiles of `tile` rays from ray 0.
// Either way every ray takes the same near lenses with the same arithmetic
// (a straddling wave's lanes give the lenses outside their own cells mass 0).
std::vector<TileSpan> make_tiles(const irs_geometry_info &gi, int axis, int32_t tile,
                                 int32_t min_span, bool weigh)
{
    const int64_t n = axis ? gi.ny : gi.nx, ncell = axis ? gi.n1y : gi.n1x;
    std::vector<TileSpan> out;
    bool follow = true;
    int64_t slots = 0;                            // tile positions when following
    for (int64_t c = 0; c < ncell && follow; ++c) {
        int64_t a, b;
        level1_span(gi, axis, c, a, b);
        follow = b - a >= min_span;
        slots += (b - a + tile - 1) / tile * tile;
    }
    if (follow && weigh && slots > 0) {
        // following the cells leaves the lanes past a cell's last column idle;
        // fixed tiles keep every lane busy, but a tile that crosses a cell
        // boundary takes the lenses of one more cell column (4 instead of 3)
        // in its near-lens pass, which is about 0.55 of the level-3 work.  A
        // tile of `tile` columns crosses (tile - 1)/C boundaries on average.
        const double idle = 1.0 - (double)n / (double)slots;
        const double cols = (double)n / (double)ncell;
        const double extra = 0.55 * ((double)(tile - 1) / cols) / 3.0;
        follow = idle <= extra;
    }
    if (follow) {
        for (int64_t c = 0; c < ncell; ++c) {
            int64_t a, b;
            level1_span(gi, axis, c, a, b);
            for (int64_t s = a; s < b; s += tile)
                out.push_back(TileSpan{(int32_t)s, (int32_t)std::min<int64_t>(b, s + tile)});
        }
    } else {
        for (int64_t s = 0; s < n; s += tile)
            out.push_back(TileSpan{(int32_t)s, (int32_t)std::min<int64_t>(n, s + tile)});
    }
    return out;
}

// The level-3 row table and tiles (geometry only, built once per plan; the
// build waits for its kernel, so work on other streams may read them at once).
irs_status ensure_rows(irs_plan_s *p)
{
    if (p->d_rows) return IRS_OK;                 // set last: the tables are all there
    irs_status st = alloc_allowed(p, "the level-3 row table");
    if (st != IRS_OK) return st;
    const DevGeom &g = p->dg;
    // column tiles follow the cells when a cell holds >= 1.5 waves of
    // columns and the idle lanes cost less than straddling; row tiles when a
    // cell holds a whole tile of rows
    p->h_tcol = make_tiles(p->geo.info, 0, kWave, kWave + kWave / 2, true);
    p->h_trow = make_tiles(p->geo.info, 1, kL3Rows, kL3Rows, false);
    dev_free(p->d_tcol);
    dev_free(p->d_trow);
    dev_free(p->d_cols);
    p->d_tcol = p->d_trow = nullptr;
    p->d_cols = nullptr;
    IRS_HIP(dev_alloc(&p->d_tcol, p->h_tcol.size() * sizeof(TileSpan)));
    IRS_HIP(dev_alloc(&p->d_trow, p->h_trow.size() * sizeof(TileSpan)));
    IRS_HIP(hipMemcpyAsync(p->d_tcol, p->h_tcol.data(), p->h_tcol.size() * sizeof(TileSpan),
                           hipMemcpyHostToDevice, p->stream));
    IRS_HIP(hipMemcpyAsync(p->d_trow, p->h_trow.data(), p->h_trow.size() * sizeof(TileSpan),
                           hipMemcpyHostToDevice, p->stream));
    IRS_HIP(dev_alloc(&p->d_cols, (size_t)g.nx * sizeof(ColInfo)));
    hipLaunchKernelGGL(k_col_table, dim3((unsigned)((g.nx + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, p->stream, g, (ColInfo *)p->d_cols);
    IRS_HIP(hipGetLastError());
    void *rows = nullptr;
    IRS_HIP(dev_alloc(&rows, (size_t)g.ny * sizeof(RowInfo)));
    const unsigned nb = (unsigned)((g.ny + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_row_table, dim3(nb), dim3(kThreads), 0, p->stream, g, (RowInfo *)rows);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        dev_free(rows);
        return hip_fail(e, "the level-3 row and column tables");
    }
    p->d_rows = rows;
    return IRS_OK;
}

void interp_band_row_bytes(const irs_plan_s *p, int64_t &coef_row, int64_t &part_row)
{
    coef_row = level2_row_bytes(p);
    const int P = level2_order(p);
    part_row = P > 0 ? (int64_t)p->dg.n1x * level2_chunks(p) * P * 2 * (int64_t)sizeof(double) : 0;
}

irs_status interp_tables_ready(irs_plan_s *p)
{
    const char *missing = nullptr;
    if (!p->d_rows) missing = "the level-3 row table";
    else if (super_order(p) > 0) {
        const size_t whole = sizeof(double) * (size_t)super_ny(p) * super_nx(p) * lens_chunks(p) *
                             super_order(p) * 2;
        if (!p->d_super || p->super_part_bytes < whole) missing = "the super-cell expansions";
        else if (mid_side(p) > 0 && !p->d_mid) missing = "the mid-cell expansions";
    }
    if (missing) {
        set_error(std::string(missing) + " of this plan are not allocated yet (shoot one whole "
                  "map with irs_shoot_map first; it sizes the plan's tables)");
        return IRS_E_INVALID;
    }
    return IRS_OK;
}

irs_status interp_prepare(irs_plan_s *p)
{
    if (std::max(p->dg.w1, p->dg.h1) > kMaxCell) {
        set_error("level-1 cells wider than 1e24: the interpolation needs narrower cells");
        return IRS_E_INVALID;
    }
    p->coef_c0 = -1;                 // nothing resident that a replay could rely on
    p->coef_c1 = -2;
    irs_status st = ensure_rows(p);
    if (st != IRS_OK) return st;
    st = ensure_bands(p, band_rows(p));
    if (st != IRS_OK) return st;
    return level2_prepare(p);
}

// Algorithmic FP64 flops of the level-3 rays of rows [j0, j1): per ray 46
// (Horner of C_0..C_4: 32, sheet 2, macro term 6, beta 2, pixel 4) plus 10 per
// nearby lens (offsets 2, r^2 3, m/r^2 1, products 2, sums 2).
double level3_flops(irs_plan_s *p, int64_t j0, int64_t j1)
{
    const DevGeom &g = p->dg;
    if (j1 <= j0) return 0.0;
    std::vector<int64_t> &cols = p->h_cell_cols;
    if ((int64_t)cols.size() != g.n1x) {                    // ray columns of each cell column
        cols.assign(g.n1x, 0);
        for (int64_t cx = 0, i = 0; cx < g.n1x; ++cx)
            while (i < g.nx && ((2 * i + 1) * (int64_t)g.n1x) / (2 * g.nx) == cx) { ++cols[cx]; ++i; }
    }
    double f = 0.0;
    for (int64_t j = j0; j < j1;) {
        const int64_t cy = ((2 * j + 1) * (int64_t)g.n1y) / (2 * g.ny);
        int64_t jn = j;
        while (jn < j1 && ((2 * jn + 1) * (int64_t)g.n1y) / (2 * g.ny) == cy) ++jn;
        double row = 0.0;
        for (int64_t cx = 0; cx < g.n1x; ++cx) {
            const int64_t xl = std::max<int64_t>(0, cx - 1), xh = std::min<int64_t>(g.n1x - 1, cx + 1);
            int64_t nn = 0;
            for (int64_t r = std::max<int64_t>(0, cy - 1); r <= std::min<int64_t>(g.n1y - 1, cy + 1); ++r)
                nn += p->h_cell_start[r * g.n1x + xh + 1] - p->h_cell_start[r * g.n1x + xl];
            row += (double)cols[cx] * (46.0 + 10.0 * (double)nn);
        }
        f += row * (double)(jn - j);
        j = jn;
    }
    return f;
}

namespace {

// The launch arguments of a plan's level 3 over rows [jr0, jr1) with the
// coefficients resident from level-1 row cy0 (queue fields left empty).
L3Map map_args(const irs_plan_s *p, const RaySel &sel, int32_t cy0, int64_t jr0, int64_t jr1)
{
    L3Map m{};
    m.g = p->dg;
    m.lxy = (const double2 *)p->d_xy;
    m.lm = p->d_m;
    m.cell_start = p->d_cell_start;
    m.rows = (const RowInfo *)p->d_rows;
    m.cols = (const ColInfo *)p->d_cols;
    m.coef = p->d_coef;
    m.tcol = p->d_tcol;
    m.trow = p->d_trow;
    m.cy0 = cy0;
    m.ntx = (int32_t)p->h_tcol.size();
    m.jr0 = jr0;
    m.jr1 = jr1;
    m.ray_first = sel.ray_first;
    m.ray_last = sel.ray_last;
    m.a1o = sel.alpha1;
    m.a2o = sel.alpha2;
    m.pixo = sel.pixel;
    m.counts = sel.counts;
    m.landed = sel.landed;
    return m;
}

// The rectangle's corner cells that hold rays of rows [jA, jB): ray columns
// [c[0], c[1]) and rows [c[2], c[3]) each; returns their number.
int corner_blocks(const irs_plan_s *p, int64_t jA, int64_t jB, int64_t c[4][4])
{
    const DevGeom &g = p->dg;
    const irs_geometry_info &gi = p->geo.info;
    int n = 0;
    if (!g.sheet) return 0;
    const int64_t cys[2] = {0, g.n1y - 1}, cxs[2] = {0, g.n1x - 1};
    for (int a = 0; a < (g.n1y > 1 ? 2 : 1); ++a) {
        int64_t ja, jb;
        level1_span(gi, 1, cys[a], ja, jb);
        ja = std::max(ja, jA);
        jb = std::min(jb, jB);
        if (jb <= ja) continue;
        for (int b = 0; b < (g.n1x > 1 ? 2 : 1); ++b) {
            int64_t ia, ib;
            level1_span(gi, 0, cxs[b], ia, ib);
            if (ib <= ia) continue;
            c[n][0] = ia;
            c[n][1] = ib;
            c[n][2] = ja;
            c[n][3] = jb;
            ++n;
        }
    }
    return n;
}

// k_level3_corner over the rays of rows [jA, jB) in the rectangle's corner
// cells (m: the band's launch arguments)
irs_status launch_corners(irs_plan_s *p, const L3Map &m, int64_t jA, int64_t jB)
{
    int64_t c[4][4];
    const int nc = corner_blocks(p, jA, jB, c);
    const bool bin = m.counts != nullptr;
    for (int k = 0; k < nc; ++k) {
        const int64_t n = (c[k][1] - c[k][0]) * (c[k][3] - c[k][2]);
        const unsigned nb = (unsigned)((n + kThreads - 1) / kThreads);
#define IRS_L3C(U, B)                                                                        \
    hipLaunchKernelGGL((k_level3_corner<U, B>), dim3(nb), dim3(kThreads), 0, p->stream, m,   \
                       c[k][0], c[k][1], c[k][2], c[k][3])
        if (p->unit_mass) {
            if (bin) IRS_L3C(true, true);
            else IRS_L3C(true, false);
        } else {
            if (bin) IRS_L3C(false, true);
            else IRS_L3C(false, false);
        }
#undef IRS_L3C
        IRS_HIP(hipGetLastError());
    }
    return IRS_OK;
}

// The super (and mid) rows that level-1 rows [cyA, cyB] need, in one launch
// each (a band's own rows fill a fraction of the chip); bands then find them
// cached.  Each row's expansion is the same whatever the launch.
irs_status level2_tree_rows(irs_plan_s *p, int64_t cyA, int64_t cyB, CallStats *cs)
{
    if (level2_order(p) <= 0 || super_order(p) <= 0) return IRS_OK;
    hipStream_t s = p->stream;
    const int32_t ks = super_side(p), km = mid_side(p);
    if (cs) {
        irs_status st = cs->begin(s, 0);
        if (st != IRS_OK) return st;
    }
    double fl = 0.0;
    irs_status st = km > 0 ? ensure_mid_rows(p, cyA / km, cyB / km, cs ? &fl : nullptr)
                           : ensure_super_rows(p, cyA / ks, cyB / ks, cs ? &fl : nullptr);
    if (st != IRS_OK) return st;
    if (cs) {
        cs->level2_expand_flops += fl;
        cs->level2_flops += fl;
        if ((st = cs->end(s)) != IRS_OK) return st;
    }
    return IRS_OK;
}

// The level-2 coefficients of level-1 rows [c0, c1] into coef (from row c0):
// the cell expansions and the points' series, on the plan's stream.  The tree rows they need
// must be cached (level2_tree_rows).
irs_status level2_band(irs_plan_s *p, int64_t c0, int64_t c1, double *coef, CallStats *cs)
{
    const DevGeom &g = p->dg;
    hipStream_t s = p->stream;
    const int32_t nl = (int32_t)p->n_lens;
    const int64_t q = g.q;
    const int64_t row_pts = (int64_t)g.n1x * q * q;            // level-2 points per level-1 row
    const int P = level2_order(p);
    if (cs) {
        irs_status st = cs->begin(s, 0);
        if (st != IRS_OK) return st;
        cs->n_level2++;
        cs->level2_points += (c1 - c0 + 1) * row_pts;
        const std::vector<int32_t> &hc = p->h_cell_start;
        auto block = [&](int64_t cx, int64_t cy, int64_t r) {   // lenses in a (2r+1)^2 block
            const int64_t xl = std::max<int64_t>(0, cx - r), xh = std::min<int64_t>(g.n1x - 1, cx + r);
            int64_t n = 0;
            for (int64_t row = std::max<int64_t>(0, cy - r); row <= std::min<int64_t>(g.n1y - 1, cy + r); ++row)
                n += hc[row * g.n1x + xh + 1] - hc[row * g.n1x + xl];
            return n;
        };
        for (int64_t cy = c0; cy <= c1; ++cy)
            for (int64_t cx = 0; cx < g.n1x; ++cx) {
                const int64_t b3 = block(cx, cy, 1);
                cs->level2_pairs += q * q * (p->n_lens - b3);
                if (P == 0) {
                    const double f = 44.0 * (double)(q * q * (p->n_lens - b3));
                    cs->level2_flops += f;
                    cs->level2_expand_flops += f;
                } else {
                    const int64_t b7 = block(cx, cy, kRing);
                    cs->level2_flops += (double)(q * q) * (44.0 * (double)(b7 - b3) + 60.0 * P);
                }
            }
    }
    if (P == 0) {
        const unsigned nb2 = (unsigned)((c1 - c0 + 1) * g.n1x);
        if (p->unit_mass)
            hipLaunchKernelGGL(k_level2<true>, dim3(nb2), dim3(kThreads), 0, s, g, p->d_x,
                               p->d_y, p->d_m, p->d_cell_start, nl, (int32_t)c0, coef);
        else
            hipLaunchKernelGGL(k_level2<false>, dim3(nb2), dim3(kThreads), 0, s, g, p->d_x,
                               p->d_y, p->d_m, p->d_cell_start, nl, (int32_t)c0, coef);
    } else {
        const int32_t nxb = (g.n1x + kCellsPerBlock - 1) / kCellsPerBlock;
        // lens chunks (one level) are a property of the plan, so results
        // do not depend on how a map is cut into calls
        const int32_t nchunk = level2_chunks(p);
        // the sheet's series is in the cell expansions when they come
        // from the super-cell path (launch_level2_expand folds it)
        const int32_t fold = super_order(p) > 0 ? 1 : 0;
        const unsigned nbB = (unsigned)((c1 - c0 + 1) * nxb);
        double fl = 0.0;
        irs_status st3 = launch_level2_expand(p, c0, c1, cs ? &fl : nullptr, true);
        if (st3 != IRS_OK) return st3;
        if (cs) {
            cs->level2_expand_flops += fl;
            cs->level2_flops += fl;
        }
#define IRS_L2L(U, PP)                                                                        \
    do {                                                                                      \
        if (cs && (st2 = cs->end(s)) != IRS_OK) return st2;                                  \
        if (cs && (st2 = cs->begin(s, 2)) != IRS_OK) return st2;                             \
        if (ring_fits(p))                                                                     \
            hipLaunchKernelGGL((k_level2_points<U, PP, false, true>), dim3(nbB), dim3(kThreads), \
                               0, s, g, p->d_x, p->d_y, p->d_m, p->d_cell_start, (int32_t)c0, \
                               nxb, nchunk, fold, p->d_part, coef);                          \
        else                                                                                  \
            hipLaunchKernelGGL((k_level2_points<U, PP, false, false>), dim3(nbB), dim3(kThreads), \
                               0, s, g, p->d_x, p->d_y, p->d_m, p->d_cell_start, (int32_t)c0, \
                               nxb, nchunk, fold, p->d_part, coef);                          \
        if (g.sheet)                                                                          \
            hipLaunchKernelGGL((k_level2_points<U, PP, true, false>), dim3(nbB), dim3(kThreads), 0, \
                               s, g, p->d_x, p->d_y, p->d_m, p->d_cell_start, (int32_t)c0,    \
                               nxb, nchunk, fold, p->d_part, coef);                          \
    } while (0)
        irs_status st2 = IRS_OK;
        if (p->unit_mass) {
            if (P == 32) IRS_L2L(true, 32);
            else IRS_L2L(true, 48);
        } else {
            if (P == 32) IRS_L2L(false, 32);
            else IRS_L2L(false, 48);
        }
#undef IRS_L2L
    }
    IRS_HIP(hipGetLastError());
    if (cs) {
        irs_status st = cs->end(s);
        if (st != IRS_OK) return st;
    }
    return IRS_OK;
}

}  // namespace

namespace {

// Level 3 of one band of level-1 rows [c0, c1] whose coefficients are in
// coef (from level-1 row cy0), on stream s: the band's row tiles, then its
// rays in the rectangle's corner cells.
irs_status level3_band(irs_plan_s *p, const RaySel &sel, int64_t c0, int64_t c1,
                       const double *coef, int64_t cy0, hipStream_t s)
{
    const DevGeom &g = p->dg;
    const int64_t q = g.q;
    const int64_t jA = std::max(sel.row0, first_row_at(g, c0 * q));
    const int64_t jB = std::min(sel.row1, first_row_at(g, (c1 + 1) * q));
    if (jB <= jA) return IRS_OK;
    CallStats *cs = sel.stats;
    const int64_t ntx = (int64_t)p->h_tcol.size();
    const int64_t ntx_pad = (ntx + kXcds - 1) / kXcds * kXcds;
    // the row tiles that meet rows [jA, jB)
    const std::vector<TileSpan> &tr = p->h_trow;
    const int64_t ta = std::upper_bound(tr.begin(), tr.end(), jA,
                                        [](int64_t v, const TileSpan &t) { return v < t.b; }) -
                       tr.begin();
    const int64_t tb = std::lower_bound(tr.begin(), tr.end(), jB,
                                        [](const TileSpan &t, int64_t v) { return t.a < v; }) -
                       tr.begin();
    const int64_t nty = tb - ta;
    L3Map m = map_args(p, sel, (int32_t)cy0, 0, 0);
    m.coef = coef;
    // at most 2^23 workgroups (2^31 work-items) per launch: the dispatch's
    // grid size in work-items is a 32-bit number
    const int64_t max_ty = std::max<int64_t>(1, ((int64_t)1 << 23) / ntx_pad);
    for (int64_t t0 = 0; t0 < nty; t0 += max_ty) {
        const int64_t t1 = std::min(nty, t0 + max_ty);
        const unsigned nb3 = (unsigned)((t1 - t0) * ntx_pad);
        const int64_t j0 = std::max(jA, (int64_t)tr[ta + t0].a);
        const int64_t j1 = std::min(jB, (int64_t)tr[ta + t1 - 1].b);
        m.jr0 = j0;
        m.jr1 = j1;
        if (cs) {
            irs_status st = cs->begin(s, 1);
            if (st != IRS_OK) return st;
            cs->n_rays++;
            cs->ray_flops += level3_flops(p, j0, j1);
        }
#define IRS_L3(U, B)                                                                          \
    hipLaunchKernelGGL((k_level3<U, B>), dim3(nb3), dim3(kThreads), 0, s, m,                  \
                       (int32_t)(ta + t0), (int32_t)ntx_pad)
        const bool bin = sel.counts != nullptr;
        if (p->unit_mass) {
            if (bin) IRS_L3(true, true);
            else IRS_L3(true, false);
        } else {
            if (bin) IRS_L3(false, true);
            else IRS_L3(false, false);
        }
#undef IRS_L3
        IRS_HIP(hipGetLastError());
        if (t1 == nty) {
            // the band's rays in the rectangle's corner cells (launched on
            // the plan's stream, which is s here)
            irs_status st = launch_corners(p, m, jA, jB);
            if (st != IRS_OK) return st;
        }
        if (cs) {
            irs_status st = cs->end(s);
            if (st != IRS_OK) return st;
        }
    }
    return IRS_OK;
}

}  // namespace

irs_status launch_interp(irs_plan_s *p, const RaySel &sel)
{
    const DevGeom &g = p->dg;
    hipStream_t s = p->stream;
    if (sel.row1 <= sel.row0) return IRS_OK;
    const int64_t q = g.q;
    const int64_t cyA = level2_row_host(g, sel.row0) / q;
    const int64_t cyB = level2_row_host(g, sel.row1 - 1) / q;  // inclusive
    const int64_t want = cyB - cyA + 1;
    irs_status st0 = ensure_rows(p);
    if (st0 != IRS_OK) return st0;
    // bands of band_rows(p) level-1 rows (the plan's budget, or the batch
    // tuner's choice), whatever larger buffer the plan holds from earlier
    const int64_t step = std::min(band_rows(p), want);
    st0 = ensure_bands(p, step);
    if (st0 != IRS_OK) return st0;
    CallStats *cs = sel.stats;
    const bool resident = p->coef_c0 <= cyA && cyB <= p->coef_c1;
    if (!resident) {
        st0 = level2_tree_rows(p, cyA, cyB, cs);
        if (st0 != IRS_OK) return st0;
    }
    for (int64_t c0 = cyA; c0 <= cyB; c0 += step) {
        const int64_t c1 = std::min(cyB, c0 + step - 1);
        if (!(p->coef_c0 <= c0 && c1 <= p->coef_c1)) {
            // the band's level-2 coefficients are not resident: compute them
            // (the buffer holds no complete band until they are done)
            p->coef_c0 = -1;
            p->coef_c1 = -2;
            st0 = level2_band(p, c0, c1, p->d_coef, cs);
            if (st0 != IRS_OK) return st0;
            p->coef_c0 = c0;
            p->coef_c1 = c1;
        }
        st0 = level3_band(p, sel, c0, c1, p->d_coef, p->coef_c0, s);
        if (st0 != IRS_OK) return st0;
    }
    return IRS_OK;
}

// ---- a batch's level 3 as one launch over every map's tiles ------------------

size_t interp_map_args_bytes() { return sizeof(L3Map); }

int64_t interp_whole_map_bytes(const irs_plan_s *p)
{
    int64_t coef_row = 0, part_row = 0;
    interp_band_row_bytes(p, coef_row, part_row);
    return (int64_t)p->dg.n1y * (coef_row + part_row);
}

irs_status interp_prepare_whole(irs_plan_s *p)
{
    p->coef_budget = (int64_t)p->dg.n1y * level2_row_bytes(p);
    return interp_prepare(p);
}

irs_status interp_level2_whole(irs_plan_s *p)
{
    p->coef_c0 = -1;
    p->coef_c1 = -2;
    irs_status st = level2_tree_rows(p, 0, p->dg.n1y - 1, nullptr);
    if (st != IRS_OK) return st;
    st = level2_band(p, 0, p->dg.n1y - 1, p->d_coef, nullptr);
    if (st != IRS_OK) return st;
    p->coef_c0 = 0;
    p->coef_c1 = p->dg.n1y - 1;
    return IRS_OK;
}

irs_status interp_map_args(irs_plan_s *p, uint32_t *counts, unsigned long long *landed,
                           void *out)
{
    if (!p->d_rows || p->coef_rows_cap < p->dg.n1y) {
        set_error("internal: a batch map's whole-map level-2 buffers are missing");
        return IRS_E_INVALID;
    }
    RaySel sel{};
    sel.ray_first = 0;
    sel.ray_last = p->dg.nx * p->dg.ny;
    sel.counts = counts;
    sel.landed = landed;
    L3Map m = map_args(p, sel, 0, 0, p->dg.ny);
    m.nty = (int32_t)p->h_trow.size();
    m.tiles = (int64_t)m.nty * ((m.ntx + kXcds - 1) / kXcds * kXcds);
    m.ncorner = corner_blocks(p, 0, p->dg.ny, m.corner);
    m.corner_items[0] = 0;
    for (int c = 0; c < 4; ++c) {
        const int64_t rays =
            c < m.ncorner ? (m.corner[c][1] - m.corner[c][0]) * (m.corner[c][3] - m.corner[c][2])
                          : 0;
        m.corner_items[c + 1] = m.corner_items[c] + (rays + kThreads - 1) / kThreads;
    }
    *(L3Map *)out = m;
    return IRS_OK;
}

irs_status interp_maps_table(const void *args, int32_t n, void *d_maps, int64_t *d_start,
                             int64_t *d_cstart, hipStream_t s)
{
    const L3Map *maps = (const L3Map *)args;
    std::vector<int64_t> start(n + 1, 0), cstart(n + 1, 0);
    for (int32_t k = 0; k < n; ++k) {
        start[k + 1] = start[k] + maps[k].tiles;
        cstart[k + 1] = cstart[k] + maps[k].corner_items[4];
    }
    IRS_HIP(hipMemcpyAsync(d_maps, args, sizeof(L3Map) * (size_t)n, hipMemcpyHostToDevice, s));
    IRS_HIP(hipMemcpyAsync(d_start, start.data(), sizeof(int64_t) * (size_t)(n + 1),
                           hipMemcpyHostToDevice, s));
    IRS_HIP(hipMemcpyAsync(d_cstart, cstart.data(), sizeof(int64_t) * (size_t)(n + 1),
                           hipMemcpyHostToDevice, s));
    IRS_HIP(hipStreamSynchronize(s));
    return IRS_OK;
}

irs_status launch_interp_maps(hipStream_t s, bool unit, const void *args, const void *d_maps,
                              const int64_t *d_start, const int64_t *d_cstart, int32_t n)
{
    const L3Map *maps = (const L3Map *)args;
    int64_t tiles = 0, corners = 0;
    for (int32_t k = 0; k < n; ++k) {
        tiles += maps[k].tiles;
        corners += maps[k].corner_items[4];
    }
    if (tiles > 0) {
        // rows of up to 2^23 workgroups (a multiple of the XCDs; 2^31 threads)
        const int64_t gx = std::min<int64_t>((tiles + kXcds - 1) / kXcds * kXcds, 1 << 23);
        const int64_t gy = (tiles + gx - 1) / gx;
        if (gy > 65535) {
            set_error("too many level-3 tiles in one batch");
            return IRS_E_INVALID;
        }
        if (unit)
            hipLaunchKernelGGL(k_level3_maps<true>, dim3((unsigned)gx, (unsigned)gy),
                               dim3(kThreads), 0, s, (const L3Map *)d_maps, d_start, n);
        else
            hipLaunchKernelGGL(k_level3_maps<false>, dim3((unsigned)gx, (unsigned)gy),
                               dim3(kThreads), 0, s, (const L3Map *)d_maps, d_start, n);
        IRS_HIP(hipGetLastError());
    }
    if (corners > 0) {
        if (unit)
            hipLaunchKernelGGL(k_level3_maps_corners<true>, dim3((unsigned)corners),
                               dim3(kThreads), 0, s, (const L3Map *)d_maps, d_cstart, n);
        else
            hipLaunchKernelGGL(k_level3_maps_corners<false>, dim3((unsigned)corners),
                               dim3(kThreads), 0, s, (const L3Map *)d_maps, d_cstart, n);
        IRS_HIP(hipGetLastError());
    }
    return IRS_OK;
}

}  // namespace irs
