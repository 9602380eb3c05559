// Direct ray shooting: every ray sums every lens (Eq. 6), then the macro term
// and the negative sheet (the rectangle's closed forms of Appendix A, or
// -kappa_* theta on a circular lens plane, Eq. 9), the mapping
// beta = theta - alpha (Eq. 4) and the source-pixel binning.  This is the
// ordinary IRS the paper compares against (Sec. 3.1), whose cost grows as
// N_rays * N_* (Eq. 12).
//
// Two kernels:
//   k_direct_f64  -- plain double precision, one ray per lane, lens tiles in LDS.
//   k_direct_f32  -- the FP32 VALU-bound form: each workgroup owns a compact
//                    64 x 32 tile of rays; ray-lens offsets are rounded to
//                    FP32 once from their FP64 values (d1 per column and
//                    lens, d2 per row and lens through LDS), eight rays per
//                    lane share every d1, and each ray's sum is compensated:
//                    32 lenses are summed plainly, then added with Kahan's
//                    correction.  The lenses
//                    of the 3 x 3 level-1 cells around the ray are then
//                    re-evaluated in FP64 and the difference to their FP32
//                    terms is added (FP32 quantisation of a lens at distance d
//                    errs by ~1e-7/d^2, which only matters close by).  The
//                    macro term, the sheet and beta are assembled in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "plan.hpp"

namespace irs {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;

// -------------------------------------------------------------------------
// Epilogue shared by both kernels: macro term + sheet + beta + pixel.
// -------------------------------------------------------------------------
__device__ __forceinline__ void assemble(const DevGeom &g, double t1, double t2, double s1,
                                         double s2, double &a1, double &a2, int32_t &pix)
{
    double h1 = 0.0, h2 = 0.0;
    if (g.sheet == 2) {                      // circular plane: -kappa_* theta (Eq. 9)
        h1 = -g.kappa_star * t1;
        h2 = -g.kappa_star * t2;
    } else if (g.sheet) {
        double I1, I2;
        sheet_unit(g, t1, t2, I1, I2);
        const double f = -g.kappa_star / M_PI;
        h1 = f * I1;
        h2 = f * I2;
    }
    a1 = g.kpg * t1 + s1 + h1;
    a2 = g.kmg * t2 + s2 + h2;
    pix = pixel_of(g, t1 - a1, t2 - a2);
}

// Per-ray output or binning, called by every lane.
__device__ __forceinline__ void emit(bool valid, int64_t out_idx, double a1, double a2,
                                     int32_t pix, double *a1o, double *a2o, int64_t *pixo,
                                     uint32_t *counts, unsigned long long *landed)
{
    if (counts) {
        const int32_t pv = valid ? pix : -1;
        bin_wave(counts, pv);
        const uint64_t got = __ballot(pv >= 0);
        if (__lane_id() == 0 && got) landed_add(landed, (unsigned long long)__popcll(got));
    } else if (valid) {
        if (a1o) a1o[out_idx] = a1;
        if (a2o) a2o[out_idx] = a2;
        if (pixo) pixo[out_idx] = pix;
    }
}

// -------------------------------------------------------------------------
// FP64
// -------------------------------------------------------------------------
constexpr int kLens64 = 256;

template <bool UNIT>
__global__ __launch_bounds__(kThreads) void k_direct_f64(
    DevGeom g, const double *__restrict__ lx, const double *__restrict__ ly,
    const double *__restrict__ lm, int32_t nl, int64_t r_begin, int64_t r_end,
    int64_t out_base, double *a1o, double *a2o, int64_t *pixo, uint32_t *counts,
    unsigned long long *landed)
{
    __shared__ double s_x[kLens64], s_y[kLens64], s_m[UNIT ? 1 : kLens64];
    const int tid = threadIdx.x;
    const int64_t r = r_begin + (int64_t)blockIdx.x * kThreads + tid;
    const bool valid = r < r_end;
    const int64_t rr = valid ? r : r_begin;
    const double t1 = ray_x(g, rr % g.nx), t2 = ray_y(g, rr / g.nx);
    double s1 = 0.0, s2 = 0.0;
    for (int32_t base = 0; base < nl; base += kLens64) {
        __syncthreads();
        if (base + tid < nl) {
            s_x[tid] = lx[base + tid];
            s_y[tid] = ly[base + tid];
            if (!UNIT) s_m[tid] = lm[base + tid];
        }
        __syncthreads();
        const int cnt = min(kLens64, nl - base);
        for (int t = 0; t < cnt; ++t) {
            const double d1 = t1 - s_x[t], d2 = t2 - s_y[t];
            const double r2 = d1 * d1 + d2 * d2;
            if (r2 > 0.0) {
                const double w = (UNIT ? 1.0 : s_m[t]) / r2;
                s1 += w * d1;
                s2 += w * d2;
            }
        }
    }
    double a1, a2;
    int32_t pix;
    assemble(g, t1, t2, s1, s2, a1, a2, pix);
    emit(valid, r - out_base, a1, a2, pix, a1o, a2o, pixo, counts, landed);
}

// Persistent FP64 form for batches: item = 256 consecutive rays of a map.
template <bool UNIT>
__global__ __launch_bounds__(kThreads) void k_direct_f64_queue(
    const DirectArgs *__restrict__ maps, const int64_t *__restrict__ item_start, int32_t nmaps,
    unsigned long long *cursor)
{
    __shared__ double s_x[kLens64], s_y[kLens64], s_m[UNIT ? 1 : kLens64];
    __shared__ long long s_item;
    const int tid = threadIdx.x;
    const int64_t total = item_start[nmaps];
    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = (long long)atomicAdd(cursor, 1ull);
        __syncthreads();
        const int64_t item = s_item;
        if (item >= total) break;                    // every workgroup reaches this
        int lo = 0, hi = nmaps - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (item_start[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        const DirectArgs &a = maps[lo];
        const DevGeom &g = a.g;
        const int64_t r = (item - item_start[lo]) * kThreads + tid;
        const bool valid = r < g.nx * g.ny;
        const int64_t rr = valid ? r : 0;
        const double t1 = ray_x(g, rr % g.nx), t2 = ray_y(g, rr / g.nx);
        double s1 = 0.0, s2 = 0.0;
        for (int32_t base = 0; base < a.nl; base += kLens64) {
            __syncthreads();
            if (base + tid < a.nl) {
                s_x[tid] = a.lx[base + tid];
                s_y[tid] = a.ly[base + tid];
                if (!UNIT) s_m[tid] = a.lm[base + tid];
            }
            __syncthreads();
            const int cnt = min(kLens64, a.nl - base);
            for (int t = 0; t < cnt; ++t) {
                const double d1 = t1 - s_x[t], d2 = t2 - s_y[t];
                const double r2 = d1 * d1 + d2 * d2;
                if (r2 > 0.0) {
                    const double w = (UNIT ? 1.0 : s_m[t]) / r2;
                    s1 += w * d1;
                    s2 += w * d2;
                }
            }
        }
        double a1, a2;
        int32_t pix;
        assemble(g, t1, t2, s1, s2, a1, a2, pix);
        emit(valid, 0, a1, a2, pix, nullptr, nullptr, nullptr, a.counts, a.landed);
    }
}

// -------------------------------------------------------------------------
// FP32 with compensation
//
// Offsets are formed in FP64 and rounded to FP32 once: d1 = RN(theta1 - x_i)
// per (column, lens), shared by the lane's 8 rays; d2 = RN(theta2 - y_i) per
// (row, lens), computed once per workgroup into LDS and read by all 64
// columns as broadcasts.  A single rounding of the exact offset is unbiased;
// a tile-local frame (d1 = RN(xr - RN(x_i - o))) is not: its second rounding
// carries the ray's offset identically into every lens of a binade, which
// adds up coherently over 1e6 lenses.
// -------------------------------------------------------------------------
constexpr int kTX = kWave;            // ray columns per tile: one per lane
constexpr int kChunk = 32;            // lenses per uncompensated partial sum
constexpr float kTiny = 1e-30f;       // keeps 1/r^2 finite for a lens on a ray

// 1/r^2 from d1^2 (+ kTiny, precomputed) and d2: hardware reciprocal refined
// by one Newton step, so the result is correctly rounded and unbiased.  A
// lens on the ray gives r^2 = kTiny and a zero term (its offsets are 0).
__device__ __forceinline__ float inv_r2(float d1sq, float d2)
{
    const float r2 = fmaf(d2, d2, d1sq);
    const float v = __builtin_amdgcn_rcpf(r2);
    const float e = fmaf(-r2, v, 1.0f);
    return fmaf(v, e, v);
}

__device__ __forceinline__ void kahan_add(float &s, float &c, float x)
{
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

}  // namespace

// The FP32 tile: RPT ray rows per lane (RPT * 4 rows per tile), LT lenses per
// LDS stage.  Every shape computes each ray with the same operations in the
// same order (LT is a multiple of kChunk), so all shapes give identical bits.
template <bool UNIT, int RPT, int LT>
struct DirectTile {
    static constexpr int TY = RPT * kWaves;
    struct Smem {
        double X[LT], Y[LT];
        float4 m4[UNIT ? 1 : LT / 4];
        float4 d24[TY][LT / 4];          // d2 per (tile row, lens)
    };

    __device__ static void run(Smem &sm, const DirectArgs &a, int64_t tx, int64_t ty)
    {
        const DevGeom &g = a.g;
        {
            // skip a tile none of whose rays is asked for (block-uniform)
            const int64_t jA = max(ty * TY, a.row0), jB = min(ty * TY + TY - 1, a.row1 - 1);
            const int64_t iA = tx * kTX, iB = min(tx * kTX + kTX - 1, g.nx - 1);
            if (jA > jB || jB * g.nx + iB < a.ray_first || jA * g.nx + iA >= a.ray_last) return;
        }
        float *s_m = reinterpret_cast<float *>(sm.m4);
        const int tid = threadIdx.x;
        const int lane = tid % kWave, wave = tid / kWave;
        const int64_t i = tx * kTX + lane;
        const double t1 = ray_x(g, i);
        const int32_t nl = a.nl;

        float in1[RPT], in2[RPT], s1[RPT], c1[RPT], s2[RPT], c2[RPT];
#pragma unroll
        for (int k = 0; k < RPT; ++k) in1[k] = in2[k] = s1[k] = c1[k] = s2[k] = c2[k] = 0.0f;

        for (int32_t base = 0; base < nl; base += LT) {
            __syncthreads();
            for (int t = tid; t < LT; t += kThreads) {
                const int32_t li = base + t;
                if (li < nl) {
                    sm.X[t] = a.lx[li];
                    sm.Y[t] = a.ly[li];
                    if (!UNIT) s_m[t] = (float)a.lm[li];
                }
            }
            __syncthreads();
            const int cnt = min(LT, nl - base);
            for (int e = tid; e < TY * LT; e += kThreads) {
                const int row = e / LT, t = e % LT;
                if (t < cnt) {
                    const double t2r = ray_y(g, ty * TY + row);
                    reinterpret_cast<float *>(sm.d24[row])[t] = (float)(t2r - sm.Y[t]);
                }
            }
            __syncthreads();
            const int full = cnt - cnt % kChunk;
            for (int c = 0; c < full; c += kChunk) {
#pragma unroll 2
                for (int t = 0; t < kChunk; t += 4) {
                    float d1[4], d1sq[4], ms[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        d1[u] = (float)(t1 - sm.X[c + t + u]);
                        d1sq[u] = fmaf(d1[u], d1[u], kTiny);
                        ms[u] = UNIT ? 1.0f : s_m[c + t + u];
                    }
#pragma unroll
                    for (int k = 0; k < RPT; ++k) {
                        const float4 D = sm.d24[wave * RPT + k][(c + t) / 4];
                        const float d2s[4] = {D.x, D.y, D.z, D.w};
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            float w = inv_r2(d1sq[u], d2s[u]);
                            if (!UNIT) w = ms[u] * w;
                            in1[k] = fmaf(d1[u], w, in1[k]);
                            in2[k] = fmaf(d2s[u], w, in2[k]);
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    kahan_add(s1[k], c1[k], in1[k]);
                    kahan_add(s2[k], c2[k], in2[k]);
                    in1[k] = in2[k] = 0.0f;
                }
            }
            if (full < cnt) {
                for (int t = full; t < cnt; ++t) {
                    const float d1 = (float)(t1 - sm.X[t]);
                    const float d1sq = fmaf(d1, d1, kTiny);
                    const float m = UNIT ? 1.0f : s_m[t];
#pragma unroll
                    for (int k = 0; k < RPT; ++k) {
                        const float d2 = reinterpret_cast<const float *>(sm.d24[wave * RPT + k])[t];
                        float w = inv_r2(d1sq, d2);
                        if (!UNIT) w = m * w;
                        in1[k] = fmaf(d1, w, in1[k]);
                        in2[k] = fmaf(d2, w, in2[k]);
                    }
                }
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    kahan_add(s1[k], c1[k], in1[k]);
                    kahan_add(s2[k], c2[k], in2[k]);
                    in1[k] = in2[k] = 0.0f;
                }
            }
        }

        // FP64 near-lens residual, assembly and output, ray by ray
        const int64_t cx = ((2 * i + 1) * (int64_t)g.n1x) / (2 * g.nx);
        const int64_t cxl = cx > 0 ? cx - 1 : 0;
        const int64_t cxh = cx < g.n1x - 1 ? cx + 1 : g.n1x - 1;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int64_t j = ty * TY + wave * RPT + k;
            const int64_t r = j * g.nx + i;
            const bool valid = i < g.nx && j >= a.row0 && j < a.row1 && r >= a.ray_first &&
                               r < a.ray_last;
            const double t2 = ray_y(g, j);
            double sum1 = (double)s1[k] - (double)c1[k];
            double sum2 = (double)s2[k] - (double)c2[k];
            if (valid) {
                const int64_t cy = ((2 * j + 1) * (int64_t)g.n1y) / (2 * g.ny);
                const int64_t cyl = cy > 0 ? cy - 1 : 0;
                const int64_t cyh = cy < g.n1y - 1 ? cy + 1 : g.n1y - 1;
                double r1 = 0.0, r2s = 0.0;
                for (int64_t row = cyl; row <= cyh; ++row) {
                    const int32_t pb = a.cell_start[row * g.n1x + cxl];
                    const int32_t pe = a.cell_start[row * g.n1x + cxh + 1];
                    for (int32_t pl = pb; pl < pe; ++pl) {
                        const double X = a.lx[pl], Y = a.ly[pl];
                        const double m64 = UNIT ? 1.0 : a.lm[pl];
                        // the FP32 term exactly as the main loop formed it
                        const float d1f = (float)(t1 - X);
                        const float d2f = (float)(t2 - Y);
                        float w = inv_r2(fmaf(d1f, d1f, kTiny), d2f);
                        if (!UNIT) w = (float)m64 * w;
                        // the FP64 term
                        const double e1 = t1 - X, e2 = t2 - Y;
                        const double rr2 = e1 * e1 + e2 * e2;
                        const double w64 = rr2 > 0.0 ? m64 / rr2 : 0.0;
                        r1 += w64 * e1 - (double)d1f * (double)w;
                        r2s += w64 * e2 - (double)d2f * (double)w;
                    }
                }
                sum1 += r1;
                sum2 += r2s;
            }
            double a1, a2;
            int32_t pix;
            assemble(g, t1, t2, sum1, sum2, a1, a2, pix);
            emit(valid, r - a.ray_first, a1, a2, pix, a.a1o, a.a2o, a.pixo, a.counts, a.landed);
        }
    }
};

namespace {

template <bool UNIT, int RPT, int LT>
__global__ __launch_bounds__(kThreads) void k_direct_f32(DirectArgs a, int64_t ntx, int64_t ty0)
{
    using T = DirectTile<UNIT, RPT, LT>;
    __shared__ typename T::Smem sm;
    T::run(sm, a, (int64_t)blockIdx.x % ntx, ty0 + (int64_t)blockIdx.x / ntx);
}

// Persistent form for batches: workgroups pull (map, tile) items from a
// device queue until it is empty.  Items are numbered map by map in the
// order the host chose (longest-processing-time first); item_start[m] is the
// first item of map m and item_start[nmaps] the total.
template <bool UNIT, int RPT, int LT>
__global__ __launch_bounds__(kThreads) void k_direct_f32_queue(
    const DirectArgs *__restrict__ maps, const int64_t *__restrict__ item_start, int32_t nmaps,
    unsigned long long *cursor)
{
    using T = DirectTile<UNIT, RPT, LT>;
    __shared__ typename T::Smem sm;
    __shared__ long long s_item;
    const int64_t total = item_start[nmaps];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (long long)atomicAdd(cursor, 1ull);
        __syncthreads();
        const int64_t item = s_item;
        if (item >= total) break;                    // every workgroup reaches this
        int lo = 0, hi = nmaps - 1;                  // map m with item_start[m] <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (item_start[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        const DirectArgs &a = maps[lo];
        const int64_t t = item - item_start[lo];
        T::run(sm, a, t % a.ntx, a.ty0 + t / a.ntx);
    }
}

}  // namespace

irs_status launch_direct(irs_plan_s *p, const RaySel &sel)
{
    const DevGeom &g = p->dg;
    const int32_t nl = (int32_t)p->n_lens;
    hipStream_t s = p->stream;
    const bool unit = p->unit_mass;
    if (sel.row1 <= sel.row0) return IRS_OK;

    if (p->params.precision == IRS_FP64) {
        const int64_t rb = std::max(sel.row0 * g.nx, sel.ray_first);
        const int64_t re = std::min(sel.row1 * g.nx, sel.ray_last);
        const int64_t chunk = (int64_t)kThreads << 22;   // rays per launch
        if (sel.stats) sel.stats->direct_pairs += std::max<int64_t>(0, re - rb) * (int64_t)nl;
        for (int64_t c0 = rb; c0 < re; c0 += chunk) {
            const int64_t c1 = std::min(re, c0 + chunk);
            const unsigned nb = (unsigned)((c1 - c0 + kThreads - 1) / kThreads);
            if (sel.stats) {
                irs_status st = sel.stats->begin(s, 1);
                if (st != IRS_OK) return st;
                sel.stats->n_rays++;
            }
            if (unit)
                hipLaunchKernelGGL(k_direct_f64<true>, dim3(nb), dim3(kThreads), 0, s, g, p->d_x,
                                   p->d_y, p->d_m, nl, c0, c1, sel.ray_first, sel.alpha1,
                                   sel.alpha2, sel.pixel, sel.counts, sel.landed);
            else
                hipLaunchKernelGGL(k_direct_f64<false>, dim3(nb), dim3(kThreads), 0, s, g,
                                   p->d_x, p->d_y, p->d_m, nl, c0, c1, sel.ray_first,
                                   sel.alpha1, sel.alpha2, sel.pixel, sel.counts, sel.landed);
            IRS_HIP(hipGetLastError());
            if (sel.stats) {
                irs_status st = sel.stats->end(s);
                if (st != IRS_OK) return st;
            }
        }
        return IRS_OK;
    }

    const int v = p->direct_variant;
    const int64_t TY = direct_variant_rows(v);
    const int64_t ntx = (g.nx + kTX - 1) / kTX;
    const int64_t ty_lo = sel.row0 / TY;
    const int64_t ty_hi = (sel.row1 - 1) / TY;          // inclusive
    const int64_t max_rows_of_tiles = std::max<int64_t>(1, ((int64_t)1 << 22) / ntx);
    if (sel.stats) {
        const int64_t r0 = std::max(sel.row0 * g.nx, sel.ray_first);
        const int64_t r1 = std::min(sel.row1 * g.nx, sel.ray_last);
        sel.stats->direct_pairs += std::max<int64_t>(0, r1 - r0) * (int64_t)nl;
    }
    DirectArgs a{};
    a.g = g;
    a.lx = p->d_x;
    a.ly = p->d_y;
    a.lm = p->d_m;
    a.cell_start = p->d_cell_start;
    a.nl = nl;
    a.ntx = ntx;
    a.row0 = sel.row0;
    a.row1 = sel.row1;
    a.ray_first = sel.ray_first;
    a.ray_last = sel.ray_last;
    a.a1o = sel.alpha1;
    a.a2o = sel.alpha2;
    a.pixo = sel.pixel;
    a.counts = sel.counts;
    a.landed = sel.landed;
    for (int64_t t0 = ty_lo; t0 <= ty_hi; t0 += max_rows_of_tiles) {
        const int64_t t1 = std::min(ty_hi + 1, t0 + max_rows_of_tiles);
        const unsigned nb = (unsigned)((t1 - t0) * ntx);
        if (sel.stats) {
            irs_status st = sel.stats->begin(s, 1);
            if (st != IRS_OK) return st;
            sel.stats->n_rays++;
        }
#define IRS_DF32(U, R, L) hipLaunchKernelGGL((k_direct_f32<U, R, L>), dim3(nb), dim3(kThreads), 0, s, a, ntx, t0)
        if (unit) {
            if (v == 0) IRS_DF32(true, 4, 512);
            else if (v == 1) IRS_DF32(true, 8, 256);
            else IRS_DF32(true, 16, 128);
        } else {
            if (v == 0) IRS_DF32(false, 4, 512);
            else if (v == 1) IRS_DF32(false, 8, 256);
            else IRS_DF32(false, 16, 128);
        }
#undef IRS_DF32
        IRS_HIP(hipGetLastError());
        if (sel.stats) {
            irs_status st = sel.stats->end(s);
            if (st != IRS_OK) return st;
        }
    }
    return IRS_OK;
}

int direct_variant_rows(int v) { return (v == 0 ? 4 : v == 1 ? 8 : 16) * kWaves; }

const char *direct_variant_name(int v)
{
    return v == 0 ? "rpt4_lt512" : v == 1 ? "rpt8_lt256" : "rpt16_lt128";
}

int64_t direct_items(const irs_plan_s *p, int variant)
{
    const DevGeom &g = p->dg;
    if (p->params.precision == IRS_FP64) return (g.nx * g.ny + kThreads - 1) / kThreads;
    const int64_t TY = direct_variant_rows(variant);
    return ((g.nx + kTX - 1) / kTX) * ((g.ny + TY - 1) / TY);
}

DirectArgs direct_args_full(const irs_plan_s *p, int variant, uint32_t *counts,
                            unsigned long long *landed)
{
    DirectArgs a{};
    a.g = p->dg;
    a.lx = p->d_x;
    a.ly = p->d_y;
    a.lm = p->d_m;
    a.cell_start = p->d_cell_start;
    a.nl = (int32_t)p->n_lens;
    a.ntx = (p->dg.nx + kTX - 1) / kTX;
    a.ty0 = 0;
    a.row0 = 0;
    a.row1 = p->dg.ny;
    a.ray_first = 0;
    a.ray_last = p->dg.nx * p->dg.ny;
    a.counts = counts;
    a.landed = landed;
    (void)variant;
    return a;
}

irs_status launch_direct_queue(hipStream_t s, int precision, bool unit, int v,
                               const DirectArgs *maps, const int64_t *item_start,
                               int32_t nmaps, unsigned long long *cursor, int blocks)
{
    if (precision == IRS_FP64) {
        if (unit)
            hipLaunchKernelGGL(k_direct_f64_queue<true>, dim3(blocks), dim3(kThreads), 0, s,
                               maps, item_start, nmaps, cursor);
        else
            hipLaunchKernelGGL(k_direct_f64_queue<false>, dim3(blocks), dim3(kThreads), 0, s,
                               maps, item_start, nmaps, cursor);
    } else {
#define IRS_DQ(U, R, L) hipLaunchKernelGGL((k_direct_f32_queue<U, R, L>), dim3(blocks), dim3(kThreads), 0, s, maps, item_start, nmaps, cursor)
        if (unit) {
            if (v == 0) IRS_DQ(true, 4, 512);
            else if (v == 1) IRS_DQ(true, 8, 256);
            else IRS_DQ(true, 16, 128);
        } else {
            if (v == 0) IRS_DQ(false, 4, 512);
            else if (v == 1) IRS_DQ(false, 8, 256);
            else IRS_DQ(false, 16, 128);
        }
#undef IRS_DQ
    }
    IRS_HIP(hipGetLastError());
    return IRS_OK;
}

namespace {
__global__ void k_zero(uint32_t *__restrict__ p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}
}  // namespace

irs_status launch_zero(hipStream_t s, void *ptr, size_t n_words)
{
    if (n_words == 0) return IRS_OK;
    const size_t blocks = std::min<size_t>((n_words + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)ptr, n_words);
    IRS_HIP(hipGetLastError());
    return IRS_OK;
}

}  // namespace irs
