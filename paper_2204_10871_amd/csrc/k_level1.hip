// Level-1 packing of the lenses (flow chart of Sec. 2.4, "Lenses packed into
// level-1 grids"): every lens gets the index of the level-1 cell holding it,
// the lenses are stably sorted by that index (so a cell's lenses keep their
// input order and every run is bitwise reproducible), and cell_start[c] is
// the first sorted lens of cell c.  The sorted FP64 arrays are what every
// later kernel reads: the direct sum streams them in order, the near/far
// split of the interpolation uses cell_start.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

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

// cell_start[c] = number of sorted keys < c, for c in [0, ncell].
__global__ void k_cell_start(const int32_t *__restrict__ skey, int32_t n, int32_t ncell,
                             int32_t *__restrict__ cell_start)
{
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > ncell) return;
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (skey[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    cell_start[c] = lo;
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

    IRS_HIP(hipMalloc(&p->d_cell_start, sizeof(int32_t) * (size_t)(ncell + 1)));
    p->h_cell_start.assign((size_t)ncell + 1, 0);
    if (n == 0) {
        IRS_HIP(hipMemsetAsync(p->d_cell_start, 0, sizeof(int32_t) * (size_t)(ncell + 1), s));
        IRS_HIP(hipStreamSynchronize(s));
        return IRS_OK;
    }
    const size_t nb = sizeof(double) * (size_t)n;
    IRS_HIP(hipMalloc(&p->d_x, nb));
    IRS_HIP(hipMalloc(&p->d_y, nb));
    if (hm) IRS_HIP(hipMalloc(&p->d_m, nb));
    IRS_HIP(hipMalloc(&p->d_cxy, sizeof(uint32_t) * (size_t)n));
    IRS_HIP(hipMalloc(&p->d_xy, 2 * nb));

    double *ux = nullptr, *uy = nullptr, *um = nullptr;
    int32_t *key = nullptr, *skey = nullptr, *idx = nullptr, *perm = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    irs_status st = IRS_OK;
    int end_bit = 1;
    while (end_bit < 31 && ((int64_t)1 << end_bit) <= ncell) ++end_bit;

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

    IRS_TRY(hipMalloc(&ux, nb));
    IRS_TRY(hipMalloc(&uy, nb));
    if (hm) IRS_TRY(hipMalloc(&um, nb));
    IRS_TRY(hipMalloc(&key, sizeof(int32_t) * (size_t)n));
    IRS_TRY(hipMalloc(&skey, sizeof(int32_t) * (size_t)n));
    IRS_TRY(hipMalloc(&idx, sizeof(int32_t) * (size_t)n));
    IRS_TRY(hipMalloc(&perm, sizeof(int32_t) * (size_t)n));
    IRS_TRY(hipMemcpyAsync(ux, hx, nb, hipMemcpyHostToDevice, s));
    IRS_TRY(hipMemcpyAsync(uy, hy, nb, hipMemcpyHostToDevice, s));
    if (hm) IRS_TRY(hipMemcpyAsync(um, hm, nb, hipMemcpyHostToDevice, s));

    {
        const int tb = 256;
        const int nbk = (n + tb - 1) / tb;
        hipLaunchKernelGGL(k_cell_keys, dim3(nbk), dim3(tb), 0, s, p->dg, ux, uy, n, key, idx);
        IRS_TRY(hipGetLastError());
        IRS_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, key, skey, idx, perm, n,
                                                   0, end_bit, s));
        IRS_TRY(hipMalloc(&tmp, tmp_bytes));
        IRS_TRY(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, key, skey, idx, perm, n, 0,
                                                   end_bit, s));
        hipLaunchKernelGGL(k_gather, dim3(nbk), dim3(tb), 0, s, perm, skey, ux, uy, um, n,
                           p->dg.n1x, p->d_x, p->d_y, p->d_m, p->d_cxy, (double2 *)p->d_xy);
        IRS_TRY(hipGetLastError());
        const int nbc = (ncell + 1 + tb - 1) / tb;
        hipLaunchKernelGGL(k_cell_start, dim3(nbc), dim3(tb), 0, s, skey, n, ncell,
                           p->d_cell_start);
        IRS_TRY(hipGetLastError());
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
    dev_free(skey);
    dev_free(idx);
    dev_free(perm);
    dev_free(tmp);
    return st;
}

}  // namespace irs
