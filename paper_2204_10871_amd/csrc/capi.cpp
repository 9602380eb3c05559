// C ABI of the ray-shooting library: argument checks, plan lifetime, output
// staging between host and device, and error reporting.  All arithmetic of
// the path runs in the kernels (k_level1.hip, k_direct.hip, k_interp.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "level2.hpp"

namespace irs {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

irs_status alloc_allowed(const irs_plan_s *p, const char *what)
{
    if (!p->no_alloc) return IRS_OK;
    set_error(std::string("irs_shoot_rows_noalloc: ") + what + " would have to be allocated");
    return IRS_E_INVALID;
}

// Allocations left before the one that fails (-1: none fails).
static std::atomic<int64_t> g_fail_alloc_after{-1};

// Live device allocations: address -> bytes, and their sum.
static std::mutex g_live_mu;
static std::unordered_map<void *, size_t> g_live;
static int64_t g_live_bytes = 0;

hipError_t dev_alloc_bytes(void **ptr, size_t bytes)
{
    int64_t left = g_fail_alloc_after.load();
    while (left >= 0 && !g_fail_alloc_after.compare_exchange_weak(left, left - 1)) {
    }
    if (left == 0) {                 // this one fails; the countdown is now -1
        *ptr = nullptr;
        return hipErrorOutOfMemory;
    }
    const hipError_t e = hipMalloc(ptr, bytes);
    if (e == hipSuccess && *ptr) {
        std::lock_guard<std::mutex> lock(g_live_mu);
        g_live[*ptr] = bytes;
        g_live_bytes += (int64_t)bytes;
    }
    return e;
}

void dev_free(void *ptr)
{
    if (!ptr) return;
    {
        std::lock_guard<std::mutex> lock(g_live_mu);
        auto it = g_live.find(ptr);
        if (it != g_live.end()) {
            g_live_bytes -= (int64_t)it->second;
            g_live.erase(it);
        }
    }
    (void)hipFree(ptr);
}

irs_status hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) return IRS_E_NOMEM;
    return IRS_E_DEVICE;
}

irs_status CallStats::begin(hipStream_t s, int k)
{
    if (!timed) return IRS_OK;
    hipEvent_t a, b;
    IRS_HIP(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        set_error("hipEventCreate failed");
        return IRS_E_DEVICE;
    }
    ev.push_back(a);
    ev.push_back(b);
    ev_kind.push_back(k);
    IRS_HIP(hipEventRecord(a, s));
    return IRS_OK;
}

irs_status CallStats::end(hipStream_t s)
{
    if (!timed) return IRS_OK;
    IRS_HIP(hipEventRecord(ev.back(), s));
    return IRS_OK;
}

irs_status CallStats::collect()
{
    for (size_t k = 0; k < ev_kind.size(); ++k) {
        IRS_HIP(hipEventSynchronize(ev[2 * k + 1]));
        float ms = 0.0f;
        IRS_HIP(hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
        if (ev_kind[k] == 0) { ms_level2 += ms; ms_level2_expand += ms; }
        else if (ev_kind[k] == 2) ms_level2 += ms;
        else ms_rays += ms;
    }
    return IRS_OK;
}

CallStats::~CallStats()
{
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

namespace {

DevGeom make_dev_geom(const HostGeometry &hg)
{
    const irs_geometry_info &g = hg.info;
    DevGeom d{};
    d.a1 = g.a1;
    d.a2 = g.a2;
    d.b1 = g.b1;
    d.b2 = g.b2;
    d.ray_dx = g.ray_dx;
    d.ray_dy = g.ray_dy;
    d.nx = g.nx;
    d.ny = g.ny;
    d.kappa_star = hg.kappa_star;
    d.kpg = g.kappa + hg.gamma;
    d.kmg = g.kappa - hg.gamma;
    d.half_side = 0.5 * hg.source_side;
    d.dpix = g.dpix;
    d.inv_dpix = 1.0 / g.dpix;
    d.sheet_f = -hg.kappa_star / M_PI;
    d.npix = (int32_t)hg.npix;
    d.npix_f = (double)hg.npix;
    d.sheet = hg.sheet ? (hg.circle ? 2 : 1) : 0;
    d.n1x = (int32_t)g.n1x;
    d.n1y = (int32_t)g.n1y;
    d.q = (int32_t)g.q;
    d.w1 = (g.a2 - g.a1) / (double)g.n1x;
    d.h1 = (g.b2 - g.b1) / (double)g.n1y;
    d.w2 = (g.a2 - g.a1) / (double)(g.n1x * g.q);
    d.h2 = (g.b2 - g.b1) / (double)(g.n1y * g.q);
    return d;
}

void release(irs_plan_s *p)
{
    if (!p) return;
    dev_free(p->d_x);
    dev_free(p->d_y);
    dev_free(p->d_m);
    dev_free(p->d_cell_start);
    dev_free(p->d_cxy);
    dev_free(p->d_order);
    dev_free(p->d_xy);
    dev_free(p->d_rows);
    dev_free(p->d_cols);
    dev_free(p->d_tcol);
    dev_free(p->d_trow);
    dev_free(p->d_coef);
    dev_free(p->d_part);
    dev_free(p->d_super);
    dev_free(p->d_mid);
    dev_free(p->d_super_part);
    dev_free(p->d_counts);
    dev_free(p->d_tmp);
    dev_free(p->d_landed);
    learn_release(p);
    delete p;
}

irs_status ensure_tmp(irs_plan_s *p, size_t bytes)
{
    if (p->tmp_bytes >= bytes) return IRS_OK;
    dev_free(p->d_tmp);
    p->d_tmp = nullptr;
    p->tmp_bytes = 0;
    IRS_HIP(dev_alloc(&p->d_tmp, bytes));
    p->tmp_bytes = bytes;
    return IRS_OK;
}

irs_status run(irs_plan_s *p, const RaySel &sel)
{
    if (p->params.method == IRS_DIRECT) return launch_direct(p, sel);
    if (p->params.method == IRS_LEARNED) return launch_learned(p, sel);
    return launch_interp(p, sel);
}

// Scratch of irs_shoot_rows_noalloc: device memory the library never
// allocates at run time.  Each GPU the library runs on holds its own copy
// until the process ends.  Layout: the landed-ray counters (kLandedSlots
// 64-bit words) at offset 0; from kScratchBandOffset, the level-2 coefficient
// band followed by the cell expansions of an interpolated plan.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr size_t kScratchBandOffset = 4096;
static_assert(kLandedSlots * sizeof(unsigned long long) <= kScratchBandOffset, "scratch layout");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<char *> g_scratch_dev;    // device address of `scratch`, per device

// Device address of `scratch` on `device` (the current device), looked up
// once per device.  Host code uses only this address, never the array's name.
irs_status scratch_address(int device, char **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize((size_t)device + 1, nullptr);
    if (!g_scratch_dev[device]) {
        void *ptr = nullptr;
        IRS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_dev[device] = (char *)ptr;
    }
    *out = g_scratch_dev[device];
    return IRS_OK;
}

// While alive: the plan allocates nothing, and an interpolated plan's
// coefficient band and cell expansions live in the scratch (bands of
// band_rows level-1 rows); afterwards the plan's own buffers are back,
// unchanged.
struct NoAllocScope {
    irs_plan_s *p;
    double *coef;
    int64_t cap, c0, c1, budget;
    double *part;
    size_t part_bytes;
    NoAllocScope(irs_plan_s *plan, char *band, int64_t band_rows, int64_t coef_row,
                 int64_t part_row)
        : p(plan), coef(plan->d_coef), cap(plan->coef_rows_cap), c0(plan->coef_c0),
          c1(plan->coef_c1), budget(plan->coef_budget), part(plan->d_part),
          part_bytes(plan->part_bytes)
    {
        p->no_alloc = true;
        if (band) {
            p->d_coef = (double *)band;
            p->coef_rows_cap = band_rows;
            p->coef_c0 = -1;
            p->coef_c1 = -2;
            p->coef_budget = band_rows * coef_row;
            p->d_part = part_row > 0 ? (double *)(band + band_rows * coef_row) : nullptr;
            p->part_bytes = (size_t)(band_rows * part_row);
        }
    }
    ~NoAllocScope()
    {
        p->no_alloc = false;
        p->d_coef = coef;
        p->coef_rows_cap = cap;
        p->coef_c0 = c0;
        p->coef_c1 = c1;
        p->coef_budget = budget;
        p->d_part = part;
        p->part_bytes = part_bytes;
    }
};

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st)
    {
        if (hipEventCreate(&a) != hipSuccess) a = nullptr;
        if (a && hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            a = b = nullptr;
        }
        if (a) (void)hipEventRecord(a, s);
    }
    double stop()
    {
        float ms = 0.0f;
        if (a && hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess)
            (void)hipEventElapsedTime(&ms, a, b);
        return ms;
    }
    ~Timer()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace
}  // namespace irs

using namespace irs;

extern "C" {

const char *irs_last_error(void) { return g_last_error.c_str(); }

irs_status irs_debug_fail_alloc(int64_t after)
{
    g_fail_alloc_after.store(after < 0 ? -1 : after);
    return IRS_OK;
}

irs_status irs_debug_live_allocs(int64_t *count, int64_t *bytes)
{
    if (!count || !bytes) {
        set_error("irs_debug_live_allocs: NULL argument");
        return IRS_E_INVALID;
    }
    std::lock_guard<std::mutex> lock(g_live_mu);
    *count = (int64_t)g_live.size();
    *bytes = g_live_bytes;
    return IRS_OK;
}

irs_status irs_geometry(const irs_params *params, int64_t n_lens, irs_geometry_info *out)
{
    if (!params || !out) {
        set_error("irs_geometry: NULL argument");
        return IRS_E_INVALID;
    }
    HostGeometry hg;
    std::string err;
    const irs_status st = derive_geometry(*params, n_lens, hg, err);
    if (st != IRS_OK) {
        set_error("irs_geometry: " + err);
        return st;
    }
    *out = hg.info;
    set_error("");
    return IRS_OK;
}

irs_status irs_level1_span(const irs_geometry_info *geo, int32_t axis, int64_t c,
                           int64_t *first, int64_t *last)
{
    if (!geo || !first || !last || (axis != 0 && axis != 1)) {
        set_error("irs_level1_span: NULL argument or axis not 0/1");
        return IRS_E_INVALID;
    }
    const int64_t nc = axis ? geo->n1y : geo->n1x;
    if (c < 0 || c >= nc || geo->q < 1 || geo->nx < 1 || geo->ny < 1) {
        set_error("irs_level1_span: level-1 index outside the grid");
        return IRS_E_INVALID;
    }
    level1_span(*geo, axis, c, *first, *last);
    set_error("");
    return IRS_OK;
}

irs_status irs_source_side(const irs_params *params, int64_t n_star, double *source_side)
{
    if (!params || !source_side || n_star < 1) {
        set_error("irs_source_side: NULL argument or n_star < 1");
        return IRS_E_INVALID;
    }
    std::string err;
    const irs_status st = source_side_for_lens_count(*params, n_star, *source_side, err);
    if (st != IRS_OK) {
        set_error("irs_source_side: " + err);
        return st;
    }
    set_error("");
    return IRS_OK;
}

irs_status irs_plan(const irs_params *params, int64_t n_lens, const double *x, const double *y,
                    const double *m, void *hip_stream, irs_plan_t *out)
{
    if (out) *out = nullptr;
    if (!params || !out || (n_lens > 0 && (!x || !y))) {
        set_error("irs_plan: NULL argument");
        return IRS_E_INVALID;
    }
    HostGeometry hg;
    std::string err;
    irs_status st = derive_geometry(*params, n_lens, hg, err);
    if (st != IRS_OK) {
        set_error("irs_plan: " + err);
        return st;
    }
    double msum = 0.0;
    for (int64_t i = 0; i < n_lens; ++i) {
        if (!std::isfinite(x[i]) || !std::isfinite(y[i]) || (m && !(std::isfinite(m[i]) && m[i] >= 0.0))) {
            set_error("irs_plan: lens positions must be finite and masses finite and >= 0");
            return IRS_E_INVALID;
        }
        msum += m ? m[i] : 1.0;
    }
    if (params->method != IRS_DIRECT && n_lens > 0) {
        // the distant-field series hold for lenses inside their level-1 cells
        const irs_geometry_info &gi = hg.info;
        const double tol = 1e-6 * std::min(gi.ix / gi.n1x, gi.iy / gi.n1y);
        for (int64_t i = 0; i < n_lens; ++i) {
            if (x[i] < gi.a1 - tol || x[i] > gi.a2 + tol || y[i] < gi.b1 - tol ||
                y[i] > gi.b2 + tol) {
                set_error("irs_plan: the interpolated methods need every lens inside the lens "
                          "rectangle [a1, a2] x [b1, b2]");
                return IRS_E_INVALID;
            }
        }
    }
    irs_plan_s *p = new (std::nothrow) irs_plan_s();
    if (!p) {
        set_error("irs_plan: host allocation failed");
        return IRS_E_NOMEM;
    }
    p->params = *params;
    p->geo = hg;
    p->dg = make_dev_geom(hg);
    p->stream = (hipStream_t)hip_stream;
    p->n_lens = n_lens;
    p->unit_mass = (m == nullptr);
    p->kappa_star_eff = M_PI * msum / (hg.info.ix * hg.info.iy);
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        st = hip_fail(e, "hipGetDevice");
        release(p);
        return st;
    }
    e = dev_alloc(&p->d_landed, sizeof(unsigned long long) * kLandedSlots);
    if (e != hipSuccess) {
        st = hip_fail(e, "hipMalloc");
        release(p);
        return st;
    }
    st = pack_level1(p, x, y, m);
    if (st != IRS_OK) {
        release(p);
        return st;
    }
    *out = p;
    set_error("");
    return IRS_OK;
}

irs_status irs_plan_set_direct_variant(irs_plan_t plan, int32_t variant)
{
    if (!plan || variant < 0 || variant >= kDirectVariants) {
        set_error("irs_plan_set_direct_variant: NULL plan or variant out of range");
        return IRS_E_INVALID;
    }
    plan->direct_variant = variant;
    return IRS_OK;
}

irs_status irs_plan_geometry(irs_plan_t plan, irs_geometry_info *out)
{
    if (!plan || !out) {
        set_error("irs_plan_geometry: NULL argument");
        return IRS_E_INVALID;
    }
    *out = plan->geo.info;
    return IRS_OK;
}

irs_status irs_plan_level1(irs_plan_t plan, int32_t *cell_start, int32_t *order)
{
    if (!plan || !cell_start || (plan->n_lens > 0 && !order)) {
        set_error("irs_plan_level1: NULL argument");
        return IRS_E_INVALID;
    }
    std::copy(plan->h_cell_start.begin(), plan->h_cell_start.end(), cell_start);
    if (plan->n_lens > 0) {
        IRS_HIP(hipMemcpyAsync(order, plan->d_order, sizeof(int32_t) * (size_t)plan->n_lens,
                               hipMemcpyDeviceToHost, plan->stream));
        IRS_HIP(hipStreamSynchronize(plan->stream));
    }
    set_error("");
    return IRS_OK;
}

irs_status irs_deflect_grid(irs_plan_t plan, int64_t first_ray, int64_t n, double *alpha1,
                            double *alpha2, int64_t *pixel, uint64_t flags)
{
    if (!plan) {
        set_error("irs_deflect_grid: NULL plan");
        return IRS_E_INVALID;
    }
    const irs_geometry_info &g = plan->geo.info;
    const int64_t total = g.nx * g.ny;
    if (first_ray < 0 || n < 0 || first_ray > total || n > total - first_ray) {
        set_error("irs_deflect_grid: ray range outside [0, nx*ny)");
        return IRS_E_INVALID;
    }
    if (n == 0) return IRS_OK;
    const bool on_dev = (flags & IRS_OUT_ON_DEVICE) != 0;
    CallStats cs;
    RaySel sel{};
    sel.stats = &cs;
    sel.row0 = first_ray / g.nx;
    sel.row1 = (first_ray + n - 1) / g.nx + 1;
    sel.ray_first = first_ray;
    sel.ray_last = first_ray + n;
    irs_status st;
    if (on_dev) {
        sel.alpha1 = alpha1;
        sel.alpha2 = alpha2;
        sel.pixel = pixel;
    } else {
        const size_t per = (size_t)n * sizeof(double);
        st = ensure_tmp(plan, 3 * per);
        if (st != IRS_OK) return st;
        char *base = (char *)plan->d_tmp;
        sel.alpha1 = alpha1 ? (double *)base : nullptr;
        sel.alpha2 = alpha2 ? (double *)(base + per) : nullptr;
        sel.pixel = pixel ? (int64_t *)(base + 2 * per) : nullptr;
    }
    st = run(plan, sel);
    if (st != IRS_OK) return st;
    if (!on_dev) {
        const size_t per = (size_t)n * sizeof(double);
        if (alpha1) IRS_HIP(hipMemcpyAsync(alpha1, sel.alpha1, per, hipMemcpyDeviceToHost, plan->stream));
        if (alpha2) IRS_HIP(hipMemcpyAsync(alpha2, sel.alpha2, per, hipMemcpyDeviceToHost, plan->stream));
        if (pixel) IRS_HIP(hipMemcpyAsync(pixel, sel.pixel, per, hipMemcpyDeviceToHost, plan->stream));
    }
    IRS_HIP(hipStreamSynchronize(plan->stream));
    set_error("");
    return IRS_OK;
}

static irs_status shoot(irs_plan_t plan, int64_t row0, int64_t nrows, uint32_t *counts,
                        irs_map_stats *stats, uint64_t flags, bool overwrite, const char *who)
{
    if (!plan || !counts) {
        set_error(std::string(who) + ": NULL argument");
        return IRS_E_INVALID;
    }
    const irs_geometry_info &g = plan->geo.info;
    if (row0 < 0 || nrows < 0 || row0 > g.ny || nrows > g.ny - row0) {
        set_error(std::string(who) + ": row range outside [0, ny)");
        return IRS_E_INVALID;
    }
    const bool on_dev = (flags & IRS_OUT_ON_DEVICE) != 0;
    const size_t map_bytes = sizeof(uint32_t) * (size_t)plan->geo.npix * (size_t)plan->geo.npix;
    hipStream_t s = plan->stream;
    Timer timer(s);
    uint32_t *dst = counts;
    if (!on_dev) {
        if (!plan->d_counts) IRS_HIP(dev_alloc(&plan->d_counts, map_bytes));
        dst = plan->d_counts;
    }
    if (!on_dev || overwrite) IRS_HIP(hipMemsetAsync(dst, 0, map_bytes, s));
    IRS_HIP(hipMemsetAsync(plan->d_landed, 0, sizeof(unsigned long long) * kLandedSlots, s));
    CallStats cs;
    cs.timed = (flags & IRS_TIME_PHASES) != 0;
    RaySel sel{};
    sel.stats = &cs;
    sel.row0 = row0;
    sel.row1 = row0 + nrows;
    sel.ray_first = 0;
    sel.ray_last = g.nx * g.ny;
    sel.counts = dst;
    sel.landed = plan->d_landed;
    irs_status st = run(plan, sel);
    if (st != IRS_OK) return st;
    unsigned long long slots[kLandedSlots];
    IRS_HIP(hipMemcpyAsync(slots, plan->d_landed, sizeof slots, hipMemcpyDeviceToHost, s));
    if (!on_dev) {
        std::vector<uint32_t> tmp((size_t)plan->geo.npix * (size_t)plan->geo.npix);
        IRS_HIP(hipMemcpyAsync(tmp.data(), dst, map_bytes, hipMemcpyDeviceToHost, s));
        IRS_HIP(hipStreamSynchronize(s));
        if (overwrite) std::memcpy(counts, tmp.data(), map_bytes);
        else
            for (size_t k = 0; k < tmp.size(); ++k) counts[k] += tmp[k];
    }
    IRS_HIP(hipStreamSynchronize(s));
    unsigned long long landed = 0;
    for (unsigned long long v : slots) landed += v;
    const double ms = timer.stop();
    st = cs.collect();
    if (st != IRS_OK) return st;
    if (stats) {
        stats->level2_points = cs.level2_points;
        stats->level2_pairs = cs.level2_pairs;
        stats->direct_pairs = cs.direct_pairs;
        stats->level2_flops = cs.level2_flops;
        stats->level2_expand_flops = cs.level2_expand_flops;
        stats->ms_level2_expand = cs.ms_level2_expand;
        stats->n_level2_launches = cs.n_level2;
        stats->n_ray_launches = cs.n_rays;
        stats->ms_level2 = cs.ms_level2;
        stats->ms_rays = cs.ms_rays;
        stats->ray_flops = cs.ray_flops;
        stats->rays_shot = nrows * g.nx;
        stats->rays_landed = (int64_t)landed;
        stats->rays_off = stats->rays_shot - stats->rays_landed;
        stats->n_lens = plan->n_lens;
        stats->kappa_star_eff = plan->kappa_star_eff;
        stats->ms_total = ms;
        stats->learned = (plan->params.method == IRS_LEARNED && plan->learn_ok) ? 1 : 0;
        stats->super_cells = plan->super_k;
        stats->mid_cells = plan->super_k > 0 ? plan->mid_k : 0;
    }
    set_error("");
    return IRS_OK;
}

irs_status irs_shoot_rows(irs_plan_t plan, int64_t row0, int64_t nrows, uint32_t *counts,
                          irs_map_stats *stats, uint64_t flags)
{
    return shoot(plan, row0, nrows, counts, stats, flags, false, "irs_shoot_rows");
}

irs_status irs_shoot_map(irs_plan_t plan, uint32_t *counts, irs_map_stats *stats,
                         uint64_t flags)
{
    if (!plan) {
        set_error("irs_shoot_map: NULL plan");
        return IRS_E_INVALID;
    }
    level2_reset(plan);          // a whole map computes every far-field expansion itself
    return shoot(plan, 0, plan->geo.info.ny, counts, stats, flags, true, "irs_shoot_map");
}

irs_status irs_shoot_rows_noalloc(irs_plan_t plan, int64_t row0, int64_t nrows,
                                  uint32_t *counts, int64_t *rays_landed)
{
    if (!plan || !counts) {
        set_error("irs_shoot_rows_noalloc: NULL argument");
        return IRS_E_INVALID;
    }
    const irs_geometry_info &g = plan->geo.info;
    if (row0 < 0 || nrows < 0 || row0 > g.ny || nrows > g.ny - row0) {
        set_error("irs_shoot_rows_noalloc: row range outside [0, ny)");
        return IRS_E_INVALID;
    }
    if (plan->params.method == IRS_LEARNED) {
        set_error("irs_shoot_rows_noalloc: the learned method is not provided");
        return IRS_E_UNSUPPORTED;
    }
    int device = -1;
    IRS_HIP(hipGetDevice(&device));
    if (device != plan->device) {
        set_error("irs_shoot_rows_noalloc: the plan's device must be the current device");
        return IRS_E_INVALID;
    }
    int64_t band = 0, coef_row = 0, part_row = 0;
    if (plan->params.method == IRS_INTERP) {
        interp_band_row_bytes(plan, coef_row, part_row);
        const int64_t room = (int64_t)(kScratchBytes - kScratchBandOffset);
        band = std::min<int64_t>(g.n1y, room / (coef_row + part_row));
        if (band < 1) {
            set_error("irs_shoot_rows_noalloc: one level-1 row of this plan needs " +
                      std::to_string(coef_row + part_row) + " bytes of level-2 scratch; at most " +
                      std::to_string(room) + " are available (use irs_shoot_rows)");
            return IRS_E_INVALID;
        }
        irs_status st = interp_tables_ready(plan);
        if (st != IRS_OK) return st;
    }
    char *base = nullptr;
    irs_status st = scratch_address(device, &base);
    if (st != IRS_OK) return st;
    unsigned long long *landed = (unsigned long long *)base;
    st = launch_zero(plan->stream, landed, kLandedSlots * 2);
    if (st != IRS_OK) return st;
    if (nrows > 0) {
        NoAllocScope scope(plan, band > 0 ? base + kScratchBandOffset : nullptr, band, coef_row,
                           part_row);
        RaySel sel{};
        sel.stats = nullptr;              // no timing events, no work accounting
        sel.row0 = row0;
        sel.row1 = row0 + nrows;
        sel.ray_first = 0;
        sel.ray_last = g.nx * g.ny;
        sel.counts = counts;
        sel.landed = landed;
        st = run(plan, sel);
        if (st != IRS_OK) return st;
    }
    if (rays_landed) {
        unsigned long long slots[kLandedSlots];
        IRS_HIP(hipMemcpyAsync(slots, landed, sizeof slots, hipMemcpyDeviceToHost, plan->stream));
        IRS_HIP(hipStreamSynchronize(plan->stream));
        unsigned long long sum = 0;
        for (unsigned long long v : slots) sum += v;
        *rays_landed = (int64_t)sum;
    }
    set_error("");
    return IRS_OK;
}

void irs_free(irs_plan_t plan)
{
    if (!plan) return;
    (void)hipStreamSynchronize(plan->stream);
    release(plan);
}

}  // extern "C"
