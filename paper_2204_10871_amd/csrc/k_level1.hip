// Level-1 packing of the lenses (flow chart of Sec. 2.4, "Lenses packed into
// level-1 grids"): every lens gets the index of the level-1 cell holding it,
// the lenses are stably sorted by that index (so a cell's lenses keep their
// input order and every run is bitwise reproducible), and cell_start[c] is
// the first sorted lens of cell c.  The sorted FP64 arrays are what every
// later kernel reads: the direct sum streams them in order, the near/far
// split of the interpolation uses cell_start.
//
// The sort is a least-significant-digit radix sort over 8-bit digits of the
// cell index, as many passes as the largest index needs.  Each pass counts
// the digits per block of 1024 lenses, takes the exclusive prefix sum of
// those counts in digit-major, block-minor order, and scatters every block's
// lenses to their digit's slots in input order (a lens's rank among the
// lenses of its wave with the same digit comes from ballots over the digit's
// bits), so every pass, and with it the whole sort, is stable whatever the
// distribution of lenses over the cells.  cell_start is the exclusive prefix
// sum of the per-cell counts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "plan.hpp"

namespace irs {

namespace {

__global__ void k_cell_keys(DevGeom g, const double *__restrict__ x,
                            const double *__restrict__ y, int32_t n,
                            int32_t *__restrict__ key, int32_t *__restrict__ idx)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t cx = (int64_t)floor((x[i] - g.a1) / g.w1);
    int64_t cy = (int64_t)floor((y[i] - g.b1) / g.h1);
    cx = cx < 0 ? 0 : (cx > g.n1x - 1 ? g.n1x - 1 : cx);
    cy = cy < 0 ? 0 : (cy > g.n1y - 1 ? g.n1y - 1 : cy);
    key[i] = (int32_t)(cy * g.n1x + cx);
    idx[i] = i;
}

__global__ void k_gather(const int32_t *__restrict__ perm, const int32_t *__restrict__ skey,
                         const double *__restrict__ x, const double *__restrict__ y,
                         const double *__restrict__ m, int32_t n, int32_t n1x,
                         double *__restrict__ sx, double *__restrict__ sy,
                         double *__restrict__ sm, uint32_t *__restrict__ cxy,
                         double2 *__restrict__ sxy)
{
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t i = perm[p];
    sx[p] = x[i];
    sy[p] = y[i];
    sxy[p] = make_double2(x[i], y[i]);
    if (m) sm[p] = m[i];
    const int32_t c = skey[p];
    cxy[p] = ((uint32_t)(c / n1x) << 16) | (uint32_t)(c % n1x);
}

constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;                              // elements per thread
constexpr int kScanBlock = kScanThreads * kScanPer;      // elements per block

// Exclusive prefix sum of a block's wave sums in LDS (kScanThreads / 64 of them).
__device__ __forceinline__ int32_t block_exclusive(int32_t v, int32_t *s_wave, int32_t &total)
{
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    // inclusive scan within the wave
    int32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    int32_t before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        if (w < wave) before += s_wave[w];
        total += s_wave[w];
    }
    __syncthreads();
    return before + x - v;
}

// out[i] = sum of in[j] for j < i within block i / kScanBlock; sums[b] = the
// block's total.  out may be in (each thread reads its elements before it
// writes them).
__global__ __launch_bounds__(kScanThreads) void k_scan_local(const int32_t *in,
                                                             int32_t n, int32_t *out,
                                                             int32_t *__restrict__ sums)
{
    __shared__ int32_t s_wave[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
    int32_t v[kScanPer], t = 0;
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
        v[e] = base + e < n ? in[base + e] : 0;
        t += v[e];
    }
    int32_t total;
    int32_t run = block_exclusive(t, s_wave, total);
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
        if (base + e < n) out[base + e] = run;
        run += v[e];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// exclusive prefix sum of the nb block totals in place (one workgroup)
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(int32_t *__restrict__ sums, int32_t nb)
{
    __shared__ int32_t s_wave[kScanThreads / 64];
    int32_t carry = 0;
    for (int32_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int32_t b = b0 + (int32_t)threadIdx.x;
        const int32_t v = b < nb ? sums[b] : 0;
        int32_t total;
        const int32_t ex = block_exclusive(v, s_wave, total);
        if (b < nb) sums[b] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int32_t *__restrict__ out, int32_t n,
                                                           const int32_t *__restrict__ sums)
{
    const int64_t i = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
    if (i < n) out[i] += sums[i / kScanBlock];
}

__global__ void k_cell_count(const int32_t *__restrict__ key, int32_t n, int32_t *__restrict__ cnt)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&cnt[key[i]], 1);
}

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortThreads = 256;
constexpr int kSortPer = 4;
constexpr int kSortBlock = kSortThreads * kSortPer;  // keys per block and pass
static_assert(kSortThreads == kRadix, "one digit per thread in the block tables");

// hist[d * nblk + b] = number of keys of block b whose digit at `shift` is d
__global__ __launch_bounds__(kSortThreads) void k_digit_hist(const int32_t *__restrict__ key,
                                                             int32_t n, int shift, int32_t nblk,
                                                             int32_t *__restrict__ hist)
{
    __shared__ int32_t s_cnt[kRadix];
    s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortBlock;
#pragma unroll
    for (int e = 0; e < kSortPer; ++e) {
        const int64_t i = base + (int64_t)e * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&s_cnt[(key[i] >> shift) & (kRadix - 1)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = s_cnt[threadIdx.x];
}

// Stable scatter of block b's keys (and their values) to the slots that the
// scanned table `offs` gives its digits.  The block's keys are taken in input
// order: four rounds of 256, each round wave by wave.
__global__ __launch_bounds__(kSortThreads) void k_digit_scatter(
    const int32_t *__restrict__ key_in, const int32_t *__restrict__ val_in, int32_t n, int shift,
    int32_t nblk, const int32_t *__restrict__ offs, int32_t *__restrict__ key_out,
    int32_t *__restrict__ val_out)
{
    __shared__ int32_t s_off[kRadix];
    s_off[threadIdx.x] = offs[(int64_t)threadIdx.x * nblk + blockIdx.x];
    __syncthreads();
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t base = (int64_t)blockIdx.x * kSortBlock;
    for (int e = 0; e < kSortPer; ++e) {
        const int64_t i = base + (int64_t)e * kSortThreads + threadIdx.x;
        const bool valid = i < n;
        const int32_t kv = valid ? key_in[i] : 0;
        const int32_t vv = valid ? val_in[i] : 0;
        const int d = (kv >> shift) & (kRadix - 1);
        // lanes of this wave holding a valid key with the same digit
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t set = __ballot(bit);
            same &= bit ? set : ~set;
        }
        const int32_t rank = (int32_t)__popcll(same & below);
        const bool last = (same >> lane) == 1ull;  // highest lane of its digit
        for (int w = 0; w < kSortThreads / 64; ++w) {
            if (wave == w && valid) {
                const int32_t pos = s_off[d] + rank;
                key_out[pos] = kv;
                val_out[pos] = vv;
                if (last) s_off[d] = pos + 1;
            }
            __syncthreads();
        }
    }
}

}  // namespace

irs_status pack_level1(irs_plan_s *p, const double *hx, const double *hy, const double *hm)
{
    const int32_t n = (int32_t)p->n_lens;
    const int64_t ncell64 = (int64_t)p->dg.n1x * p->dg.n1y;
    if (ncell64 >= INT32_MAX || p->dg.n1x > 65535 || p->dg.n1y > 65535) {
        set_error("level-1 grid too large (at most 65535 cells per side)");
        return IRS_E_INVALID;
    }
    const int32_t ncell = (int32_t)ncell64;
    hipStream_t s = p->stream;

    IRS_HIP(dev_alloc(&p->d_cell_start, sizeof(int32_t) * (size_t)(ncell + 1)));
    p->h_cell_start.assign((size_t)ncell + 1, 0);
    if (n == 0) {
        IRS_HIP(hipMemsetAsync(p->d_cell_start, 0, sizeof(int32_t) * (size_t)(ncell + 1), s));
        IRS_HIP(hipStreamSynchronize(s));
        return IRS_OK;
    }
    const size_t nb = sizeof(double) * (size_t)n;
    IRS_HIP(dev_alloc(&p->d_x, nb));
    IRS_HIP(dev_alloc(&p->d_y, nb));
    if (hm) IRS_HIP(dev_alloc(&p->d_m, nb));
    IRS_HIP(dev_alloc(&p->d_cxy, sizeof(uint32_t) * (size_t)n));
    IRS_HIP(dev_alloc(&p->d_xy, 2 * nb));

    double *ux = nullptr, *uy = nullptr, *um = nullptr;
    int32_t *key = nullptr, *val = nullptr, *key2 = nullptr, *val2 = nullptr;
    int32_t *cnt = nullptr, *hist = nullptr, *sums = nullptr;
    irs_status st = IRS_OK;
    const int32_t nscan = ncell + 1;  // per-cell counts then a zero: cell_start[ncell] = n
    const int32_t nblk = (n + kSortBlock - 1) / kSortBlock;
    const int32_t nhist = kRadix * nblk;
    const int32_t nsums = (std::max(nscan, nhist) + kScanBlock - 1) / kScanBlock;
    int bits = 0;
    while (bits < 31 && ((ncell - 1) >> bits) != 0) ++bits;

    auto fail = [&](hipError_t e, const char *what) {
        st = hip_fail(e, what);
    };
#define IRS_TRY(call)                                 \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) {                       \
            fail(e_, #call);                          \
            goto done;                                \
        }                                             \
    } while (0)
    // exclusive prefix sum of in[0, len) into out (three launches)
    auto scan = [&](const int32_t *in, int32_t len, int32_t *out) {
        const int32_t nb = (len + kScanBlock - 1) / kScanBlock;
        hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(kScanThreads), 0, s, in, len, out, sums);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, sums, nb);
        hipLaunchKernelGGL(k_scan_add, dim3((len + kScanThreads - 1) / kScanThreads),
                           dim3(kScanThreads), 0, s, out, len, (const int32_t *)sums);
        return hipGetLastError();
    };

    IRS_TRY(dev_alloc(&ux, nb));
    IRS_TRY(dev_alloc(&uy, nb));
    if (hm) IRS_TRY(dev_alloc(&um, nb));
    IRS_TRY(dev_alloc(&key, sizeof(int32_t) * (size_t)n));
    IRS_TRY(dev_alloc(&val, sizeof(int32_t) * (size_t)n));
    IRS_TRY(dev_alloc(&key2, sizeof(int32_t) * (size_t)n));
    IRS_TRY(dev_alloc(&val2, sizeof(int32_t) * (size_t)n));
    IRS_TRY(dev_alloc(&cnt, sizeof(int32_t) * (size_t)nscan));
    IRS_TRY(dev_alloc(&hist, sizeof(int32_t) * (size_t)nhist));
    IRS_TRY(dev_alloc(&sums, sizeof(int32_t) * (size_t)nsums));
    IRS_TRY(hipMemcpyAsync(ux, hx, nb, hipMemcpyHostToDevice, s));
    IRS_TRY(hipMemcpyAsync(uy, hy, nb, hipMemcpyHostToDevice, s));
    if (hm) IRS_TRY(hipMemcpyAsync(um, hm, nb, hipMemcpyHostToDevice, s));

    {
        const int tb = 256;
        const int nbk = (n + tb - 1) / tb;
        hipLaunchKernelGGL(k_cell_keys, dim3(nbk), dim3(tb), 0, s, p->dg, ux, uy, n, key, val);
        IRS_TRY(hipGetLastError());
        // cell_start: exclusive prefix sum of the per-cell counts
        IRS_TRY(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)nscan, s));
        hipLaunchKernelGGL(k_cell_count, dim3(nbk), dim3(tb), 0, s, key, n, cnt);
        IRS_TRY(hipGetLastError());
        IRS_TRY(scan(cnt, nscan, p->d_cell_start));
        // stable sort of (cell, lens index) pairs by cell
        for (int shift = 0; shift < bits; shift += kRadixBits) {
            hipLaunchKernelGGL(k_digit_hist, dim3(nblk), dim3(kSortThreads), 0, s, key, n, shift,
                               nblk, hist);
            IRS_TRY(hipGetLastError());
            IRS_TRY(scan(hist, nhist, hist));
            hipLaunchKernelGGL(k_digit_scatter, dim3(nblk), dim3(kSortThreads), 0, s,
                               (const int32_t *)key, (const int32_t *)val, n, shift, nblk,
                               (const int32_t *)hist, key2, val2);
            IRS_TRY(hipGetLastError());
            std::swap(key, key2);
            std::swap(val, val2);
        }
        hipLaunchKernelGGL(k_gather, dim3(nbk), dim3(tb), 0, s, val, key, ux, uy, um, n,
                           p->dg.n1x, p->d_x, p->d_y, p->d_m, p->d_cxy, (double2 *)p->d_xy);
        IRS_TRY(hipGetLastError());
        p->d_order = val;  // kept: the input index of every packed lens
        val = nullptr;
        IRS_TRY(hipMemcpyAsync(p->h_cell_start.data(), p->d_cell_start,
                               sizeof(int32_t) * (size_t)(ncell + 1), hipMemcpyDeviceToHost, s));
        IRS_TRY(hipStreamSynchronize(s));
    }
done:
#undef IRS_TRY
    dev_free(ux);
    dev_free(uy);
    dev_free(um);
    dev_free(key);
    dev_free(val);
    dev_free(key2);
    dev_free(val2);
    dev_free(cnt);
    dev_free(hist);
    dev_free(sums);
    return st;
}

}  // namespace irs
