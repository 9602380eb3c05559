// Batches of independent maps: one graph launch for all of them, with launch
// settings chosen by measurement (the autotuner) and kept in a cache file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "plan.hpp"

using namespace irs;

struct irs_batch_s {
    std::vector<irs_plan_s *> plans;       // not owned
    std::vector<int> order;                 // longest map first
    int method = 0, precision = 0;
    bool unit = true;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n_cu = 1;
    int variant = 1, bpc = 4, band_rows = 4;
    bool tuned = false, from_cache = false;
    double tune_ms = 0.0;
    // device tables of the direct queue
    DirectArgs *d_maps = nullptr;
    int64_t *d_item_start = nullptr;
    unsigned long long *d_cursor = nullptr;   // [0] cursor, then kLandedSlots landed
                                              // counters per map
    int64_t items = 0;
    // interpolated batches: every map's level 2 resident at once and level 3
    // as one launch over every map's tiles (whole), else band by band per map
    bool whole = false;
    std::vector<char> h_args;                // level-3 launch arguments, LPT order
    void *d_l3 = nullptr;                    // ... their table on the device
    int64_t *d_l3start = nullptr;            // the maps' first tiles, then all tiles
    int64_t *d_l3cstart = nullptr;           // the same for their corner-cell blocks
    // interpolated batches: parallel branches of the graph (default priority)
    std::vector<hipStream_t> lanes;
    std::vector<hipEvent_t> lane_done;
    hipEvent_t fork = nullptr;
    // captured graph
    hipGraphExec_t exec = nullptr;
    std::vector<uint32_t *> graph_counts;
    int graph_variant = -1, graph_bpc = -1, graph_band_rows = -1;
};

namespace {

constexpr int kLanes = 4;                  // parallel branches of an interpolated batch
constexpr double kWholeMemFraction = 0.6;  // of free device memory, for whole-map level 2

void drop_graph(irs_batch_s *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->graph_counts.clear();
}

double map_cost(const irs_plan_s *p)
{
    const double rays = (double)p->dg.nx * (double)p->dg.ny;
    if (p->params.method == IRS_DIRECT) return rays * (double)std::max<int64_t>(1, p->n_lens);
    const double l2 = (double)p->dg.n1x * p->dg.n1y * (double)std::max<int64_t>(1, p->n_lens);
    return rays * 40.0 + l2 * 300.0;
}

// level-2 work of a whole map (expansions of its cells against its lenses)
double map_level2_cost(const irs_plan_s *p)
{
    return (double)p->dg.n1x * p->dg.n1y * (double)std::max<int64_t>(1, p->n_lens);
}

// Tables of the direct queue for the current variant: maps in LPT order.
irs_status build_direct_tables(irs_batch_s *b, uint32_t *const *counts)
{
    const int n = (int)b->plans.size();
    std::vector<DirectArgs> maps(n);
    std::vector<int64_t> start(n + 1, 0);
    for (int k = 0; k < n; ++k) {
        const int m = b->order[k];
        irs_plan_s *p = b->plans[m];
        maps[k] = direct_args_full(p, b->variant, counts ? counts[m] : nullptr,
                                   b->d_cursor + 1 + (size_t)m * kLandedSlots);
        start[k + 1] = start[k] + direct_items(p, b->variant);
    }
    b->items = start[n];
    IRS_HIP(hipMemcpyAsync(b->d_maps, maps.data(), sizeof(DirectArgs) * n,
                           hipMemcpyHostToDevice, b->stream));
    IRS_HIP(hipMemcpyAsync(b->d_item_start, start.data(), sizeof(int64_t) * (n + 1),
                           hipMemcpyHostToDevice, b->stream));
    IRS_HIP(hipStreamSynchronize(b->stream));
    return IRS_OK;
}

// Level-3 launch arguments of every map (whole batches), LPT order, and
// their device table (before a capture: the launch reads the table).
irs_status build_map_args(irs_batch_s *b, uint32_t *const *counts)
{
    const int n = (int)b->plans.size();
    const size_t sz = interp_map_args_bytes();
    b->h_args.assign(sz * n, 0);
    for (int k = 0; k < n; ++k) {
        const int m = b->order[k];
        irs_status st = interp_map_args(b->plans[m], counts ? counts[m] : nullptr,
                                        b->d_cursor + 1 + (size_t)m * kLandedSlots,
                                        b->h_args.data() + sz * k);
        if (st != IRS_OK) return st;
    }
    return interp_maps_table(b->h_args.data(), n, b->d_l3, b->d_l3start, b->d_l3cstart,
                             b->stream);
}

// Enqueue the whole batch on b->stream (capturable: kernels only).
irs_status enqueue_all(irs_batch_s *b, uint32_t *const *counts)
{
    const int n = (int)b->plans.size();
    irs_status st = launch_zero(b->stream, b->d_cursor, 2 * (1 + (size_t)n * kLandedSlots));
    if (st != IRS_OK) return st;
    for (int m = 0; m < n; ++m) {
        const irs_plan_s *p = b->plans[m];
        st = launch_zero(b->stream, counts[m], (size_t)p->geo.npix * (size_t)p->geo.npix);
        if (st != IRS_OK) return st;
    }
    if (b->method == IRS_DIRECT)
        return launch_direct_queue(b->stream, b->precision, b->unit, b->variant, b->d_maps,
                                   b->d_item_start, n, b->d_cursor, b->bpc * b->n_cu);
    // the maps run on parallel branches (fork from the batch stream, join back);
    // longest first, each onto the branch with the least work so far.  Queue
    // batches: the branches compute the maps' level-2 fields, then one
    // launch shoots every map's tiles, longest map first.
    const int nl = (int)b->lanes.size();
    IRS_HIP(hipEventRecord(b->fork, b->stream));
    for (int l = 0; l < nl; ++l) IRS_HIP(hipStreamWaitEvent(b->lanes[l], b->fork, 0));
    std::vector<double> load(nl, 0.0);
    for (int k = 0; k < n; ++k) {
        const int m = b->order[k];
        irs_plan_s *p = b->plans[m];
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[l] += b->whole ? map_level2_cost(p) : map_cost(p);
        if (b->whole) {
            hipStream_t saved = p->stream;
            p->stream = b->lanes[l];
            st = interp_level2_whole(p);
            p->stream = saved;
            if (st != IRS_OK) return st;
            continue;
        }
        RaySel sel{};
        sel.stats = nullptr;
        sel.row0 = 0;
        sel.row1 = p->dg.ny;
        sel.ray_first = 0;
        sel.ray_last = p->dg.nx * p->dg.ny;
        sel.counts = counts[m];
        sel.landed = b->d_cursor + 1 + (size_t)m * kLandedSlots;
        hipStream_t saved = p->stream;
        p->stream = b->lanes[l];
        st = launch_interp(p, sel);
        p->stream = saved;
        if (st != IRS_OK) return st;
    }
    for (int l = 0; l < nl; ++l) {
        IRS_HIP(hipEventRecord(b->lane_done[l], b->lanes[l]));
        IRS_HIP(hipStreamWaitEvent(b->stream, b->lane_done[l], 0));
    }
    if (b->whole)
        return launch_interp_maps(b->stream, b->unit, b->h_args.data(), b->d_l3, b->d_l3start,
                                  b->d_l3cstart, n);
    return IRS_OK;
}

irs_status prepare_interp(irs_batch_s *b)
{
    if (b->whole) {
        for (irs_plan_s *p : b->plans) {
            irs_status st = interp_prepare_whole(p);
            if (st != IRS_OK) return st;
        }
        return IRS_OK;
    }
    for (irs_plan_s *p : b->plans) {
        if (b->band_rows > 0) {
            const int64_t row_bytes = (int64_t)p->dg.n1x * p->dg.q * p->dg.q * 10 * 8;
            p->coef_budget = (int64_t)b->band_rows * row_bytes;
        }
        irs_status st = interp_prepare(p);
        if (st != IRS_OK) return st;
    }
    return IRS_OK;
}

std::string tune_key(const irs_batch_s *b)
{
    const irs_plan_s *p = b->plans[b->order[0]];
    const double aspect = std::max(p->geo.info.ix, p->geo.info.iy) /
                          std::min(p->geo.info.ix, p->geo.info.iy);
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s %s %s n%d a%d",
                  b->method == IRS_DIRECT ? "direct" : "interp",
                  b->precision == IRS_FP64 ? "fp64" : "fp32", b->unit ? "unit" : "mass",
                  (int)std::lround(std::log2((double)std::max<int64_t>(1, p->n_lens))),
                  (int)std::lround(std::log2(aspect)));
    return buf;
}

bool cache_lookup(const std::string &path, const std::string &key, std::string &val)
{
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        const size_t eq = line.find(" = ");
        if (eq != std::string::npos && line.substr(0, eq) == key) {
            val = line.substr(eq + 3);
            found = true;                    // the last entry for a key wins
        }
    }
    return found;
}

void cache_store(const std::string &path, const std::string &key, const std::string &val)
{
    std::ofstream f(path, std::ios::app);
    if (f) f << key << " = " << val << "\n";
}

// time one configuration of the heaviest map (events on the batch stream)
irs_status time_direct(irs_batch_s *b, int variant, int bpc, uint32_t *scratch, double &ms)
{
    irs_plan_s *p = b->plans[b->order[0]];
    DirectArgs a = direct_args_full(p, variant, scratch, b->d_cursor + 1);
    const int64_t items = direct_items(p, variant);
    const int64_t sample = std::min<int64_t>(items, (int64_t)4 * 8 * b->n_cu);
    int64_t start[2] = {0, sample};
    IRS_HIP(hipMemcpyAsync(b->d_maps, &a, sizeof a, hipMemcpyHostToDevice, b->stream));
    IRS_HIP(hipMemcpyAsync(b->d_item_start, start, sizeof start, hipMemcpyHostToDevice, b->stream));
    EventPair ev;
    IRS_HIP(ev.create());
    const hipEvent_t e0 = ev.a, e1 = ev.b;
    irs_status st = IRS_OK;
    ms = 0.0;
    for (int rep = 0; rep < 2 && st == IRS_OK; ++rep) {     // first run warms up
        st = launch_zero(b->stream, b->d_cursor, 2 * (1 + (size_t)kLandedSlots));
        if (st == IRS_OK) st = (hipEventRecord(e0, b->stream) == hipSuccess) ? IRS_OK : IRS_E_DEVICE;
        if (st == IRS_OK)
            st = launch_direct_queue(b->stream, b->precision, b->unit, variant, b->d_maps,
                                     b->d_item_start, 1, b->d_cursor, bpc * b->n_cu);
        if (st == IRS_OK && hipEventRecord(e1, b->stream) != hipSuccess) st = IRS_E_DEVICE;
        if (st == IRS_OK && hipEventSynchronize(e1) != hipSuccess) st = IRS_E_DEVICE;
        float f = 0.0f;
        if (st == IRS_OK) (void)hipEventElapsedTime(&f, e0, e1);
        ms = (double)f * (double)items / (double)sample;     // whole-map estimate
    }
    if (st != IRS_OK) set_error("autotuner: timing launch failed");
    return st;
}

irs_status time_interp(irs_batch_s *b, int rows, uint32_t *scratch, double &ms)
{
    irs_plan_s *p = b->plans[b->order[0]];
    const int64_t row_bytes = (int64_t)p->dg.n1x * p->dg.q * p->dg.q * 10 * 8;
    p->coef_budget = (int64_t)rows * row_bytes;
    irs_status st = interp_prepare(p);
    if (st != IRS_OK) return st;
    const int64_t c1 = std::min<int64_t>(p->dg.n1y, rows) ;
    // rays of the first c1 level-1 rows
    int64_t j1 = 0;
    {
        const int64_t M = (int64_t)p->dg.n1y * p->dg.q;
        int64_t lo = 0, hi = p->dg.ny;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (((2 * mid + 1) * M) / (2 * p->dg.ny) >= c1 * p->dg.q) hi = mid;
            else lo = mid + 1;
        }
        j1 = lo;
    }
    EventPair ev;
    IRS_HIP(ev.create());
    const hipEvent_t e0 = ev.a, e1 = ev.b;
    hipStream_t saved = p->stream;
    p->stream = b->stream;
    ms = 0.0;
    for (int rep = 0; rep < 2 && st == IRS_OK; ++rep) {
        p->coef_c0 = -1;
        p->coef_c1 = -2;
        RaySel sel{};
        sel.row0 = 0;
        sel.row1 = std::max<int64_t>(1, j1);
        sel.ray_first = 0;
        sel.ray_last = p->dg.nx * p->dg.ny;
        sel.counts = scratch;
        sel.landed = b->d_cursor + 1;
        if (hipEventRecord(e0, b->stream) != hipSuccess) st = IRS_E_DEVICE;
        if (st == IRS_OK) st = launch_interp(p, sel);
        if (st == IRS_OK && hipEventRecord(e1, b->stream) != hipSuccess) st = IRS_E_DEVICE;
        if (st == IRS_OK && hipEventSynchronize(e1) != hipSuccess) st = IRS_E_DEVICE;
        float f = 0.0f;
        if (st == IRS_OK) (void)hipEventElapsedTime(&f, e0, e1);
        ms = (double)f * (double)p->dg.ny / (double)std::max<int64_t>(1, j1);
    }
    p->stream = saved;
    p->coef_c0 = -1;
    p->coef_c1 = -2;
    return st;
}

}  // namespace

extern "C" {

irs_status irs_batch_create(const irs_plan_t *plans, int32_t n, void *hip_stream,
                            irs_batch_t *out)
{
    if (out) *out = nullptr;
    if (!plans || !out || n <= 0) {
        set_error("irs_batch_create: NULL argument or empty batch");
        return IRS_E_INVALID;
    }
    for (int k = 0; k < n; ++k)
        if (!plans[k]) {
            set_error("irs_batch_create: NULL plan");
            return IRS_E_INVALID;
        }
    const irs_plan_s *p0 = plans[0];
    if (p0->params.method != IRS_DIRECT && p0->params.method != IRS_INTERP) {
        set_error("irs_batch_create: batches take IRS_DIRECT or IRS_INTERP plans");
        return IRS_E_UNSUPPORTED;
    }
    for (int k = 1; k < n; ++k) {
        const irs_plan_s *p = plans[k];
        if (p->params.method != p0->params.method || p->params.precision != p0->params.precision ||
            p->device != p0->device ||
            (p0->params.method == IRS_DIRECT && p->unit_mass != p0->unit_mass)) {
            set_error("irs_batch_create: plans differ in method, precision, device or mass kind");
            return IRS_E_UNSUPPORTED;
        }
    }
    irs_batch_s *b = new (std::nothrow) irs_batch_s();
    if (!b) {
        set_error("irs_batch_create: host allocation failed");
        return IRS_E_NOMEM;
    }
    b->plans.assign(plans, plans + n);
    b->method = p0->params.method;
    b->precision = p0->params.precision;
    b->unit = p0->unit_mass;
    b->variant = p0->direct_variant;
    b->order.resize(n);
    for (int k = 0; k < n; ++k) b->order[k] = k;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        return map_cost(b->plans[x]) > map_cost(b->plans[y]);
    });
    irs_status st = IRS_OK;
    hipError_t e = hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount,
                                         p0->device);
    if (e == hipSuccess && hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else if (e == hipSuccess) {
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        b->own_stream = (e == hipSuccess);
    }
    if (e == hipSuccess && b->method != IRS_DIRECT) {
        const int nl = std::min(n, kLanes);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        for (int l = 0; l < nl && e == hipSuccess; ++l) {
            hipStream_t ls = nullptr;
            hipEvent_t le = nullptr;
            e = hipStreamCreateWithFlags(&ls, hipStreamNonBlocking);
            if (e == hipSuccess) b->lanes.push_back(ls);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&le, hipEventDisableTiming);
            if (e == hipSuccess) b->lane_done.push_back(le);
        }
    }
    if (e == hipSuccess && b->method == IRS_INTERP) {
        // every map's level 2 at once if it fits comfortably and the maps
        // share a mass kind (one kernel instance for their level 3)
        size_t free_b = 0, total_b = 0;
        int64_t need = 0;
        bool same_mass = true;
        for (int k = 0; k < n; ++k) {
            need += interp_whole_map_bytes(plans[k]);
            same_mass = same_mass && plans[k]->unit_mass == p0->unit_mass;
        }
        e = hipMemGetInfo(&free_b, &total_b);
        const char *off = std::getenv("IRS_BATCH_BANDS");
        b->whole = e == hipSuccess && same_mass && !(off && *off && std::strcmp(off, "0") != 0) &&
                   (double)need <= kWholeMemFraction * (double)free_b;
        if (b->whole) b->band_rows = 0;
    }
    if (e == hipSuccess && b->method == IRS_INTERP) {
        e = dev_alloc(&b->d_l3, interp_map_args_bytes() * n);
        if (e == hipSuccess) e = dev_alloc(&b->d_l3start, sizeof(int64_t) * (n + 1));
        if (e == hipSuccess) e = dev_alloc(&b->d_l3cstart, sizeof(int64_t) * (n + 1));
    }
    if (e == hipSuccess) e = dev_alloc(&b->d_maps, sizeof(DirectArgs) * n);
    if (e == hipSuccess) e = dev_alloc(&b->d_item_start, sizeof(int64_t) * (n + 1));
    if (e == hipSuccess)
        e = dev_alloc(&b->d_cursor, sizeof(unsigned long long) * (1 + (size_t)n * kLandedSlots));
    if (e != hipSuccess) st = hip_fail(e, "irs_batch_create");
    if (st != IRS_OK) {
        irs_batch_free(b);
        return st;
    }
    *out = b;
    set_error("");
    return IRS_OK;
}

irs_status irs_batch_tune(irs_batch_t b, const char *cache_path)
{
    if (!b) {
        set_error("irs_batch_tune: NULL batch");
        return IRS_E_INVALID;
    }
    std::string path = cache_path ? cache_path : "";
    if (path.empty()) {
        const char *env = std::getenv("IRS_TUNE_CACHE");
        if (env) path = env;
    }
    const std::string key = tune_key(b);
    std::string val;
    if (!path.empty() && cache_lookup(path, key, val)) {
        int v = -1, bpc = -1, rows = -1;
        const int got = std::sscanf(val.c_str(), "variant=%d bpc=%d band_rows=%d", &v, &bpc,
                                    &rows);
        if (got >= 3 && v >= 0 && v < kDirectVariants && bpc > 0 && rows >= 0 &&
            (rows == 0) == b->whole) {
            b->variant = v;
            b->bpc = bpc;
            b->band_rows = rows;
            b->tuned = b->from_cache = true;
            for (irs_plan_s *p : b->plans) p->direct_variant = v;
            drop_graph(b);
            return IRS_OK;
        }
    }
    irs_plan_s *heavy = b->plans[b->order[0]];
    const size_t map_bytes = sizeof(uint32_t) * (size_t)heavy->geo.npix * (size_t)heavy->geo.npix;
    uint32_t *scratch = nullptr;
    IRS_HIP(dev_alloc(&scratch, map_bytes));
    auto t0 = std::chrono::steady_clock::now();
    irs_status st = IRS_OK;
    double best = 1e300;
    if (b->method == IRS_DIRECT && b->precision == IRS_FP32_KAHAN) {
        for (int v = 0; v < kDirectVariants && st == IRS_OK; ++v)
            for (int bpc : {2, 4, 8}) {
                double ms = 0.0;
                st = time_direct(b, v, bpc, scratch, ms);
                if (st != IRS_OK) break;
                if (ms < best) {
                    best = ms;
                    b->variant = v;
                    b->bpc = bpc;
                }
            }
    } else if (b->method == IRS_DIRECT) {
        for (int bpc : {2, 4, 8}) {
            double ms = 0.0;
            st = time_direct(b, 0, bpc, scratch, ms);
            if (st != IRS_OK) break;
            if (ms < best) {
                best = ms;
                b->bpc = bpc;
            }
        }
    } else if (b->whole) {
        // one level-3 launch of a workgroup per tile: nothing to choose
    } else {
        const int64_t n1y = heavy->dg.n1y;
        for (int rows : {1, 4, 16}) {
            if (rows > n1y && rows != 1) break;
            double ms = 0.0;
            st = time_interp(b, rows, scratch, ms);
            if (st != IRS_OK) break;
            if (ms < best) {
                best = ms;
                b->band_rows = rows;
            }
        }
    }
    dev_free(scratch);
    if (st != IRS_OK) return st;
    b->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    b->tuned = true;
    b->from_cache = false;
    for (irs_plan_s *p : b->plans) p->direct_variant = b->variant;
    drop_graph(b);
    if (!path.empty()) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "variant=%d bpc=%d band_rows=%d", b->variant, b->bpc,
                      b->band_rows);
        cache_store(path, key, buf);
    }
    set_error("");
    return IRS_OK;
}

irs_status irs_batch_run(irs_batch_t b, uint32_t *const *counts, irs_map_stats *stats,
                         uint64_t flags)
{
    (void)flags;
    if (!b || !counts) {
        set_error("irs_batch_run: NULL argument");
        return IRS_E_INVALID;
    }
    const int n = (int)b->plans.size();
    for (int k = 0; k < n; ++k)
        if (!counts[k]) {
            set_error("irs_batch_run: NULL counts pointer");
            return IRS_E_INVALID;
        }
    const bool same = b->exec && b->graph_variant == b->variant && b->graph_bpc == b->bpc &&
                      b->graph_band_rows == b->band_rows &&
                      std::equal(b->graph_counts.begin(), b->graph_counts.end(), counts);
    irs_status st = IRS_OK;
    if (!same) {
        drop_graph(b);
        if (b->method == IRS_DIRECT) st = build_direct_tables(b, counts);
        else st = prepare_interp(b);
        if (st == IRS_OK && b->whole) st = build_map_args(b, counts);
        if (st != IRS_OK) return st;
        hipGraph_t graph = nullptr;
        IRS_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        st = enqueue_all(b, counts);
        hipError_t e = hipStreamEndCapture(b->stream, &graph);
        if (st != IRS_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            b->exec = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
        b->graph_counts.assign(counts, counts + n);
        b->graph_variant = b->variant;
        b->graph_bpc = b->bpc;
        b->graph_band_rows = b->band_rows;
    }
    EventPair ev;
    hipError_t e = ev.create();
    const hipEvent_t e0 = ev.a, e1 = ev.b;
    if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
    const char *what = "irs_batch_run: timing events";
    if (e == hipSuccess) {
        e = hipGraphLaunch(b->exec, b->stream);
        what = "hipGraphLaunch";
    }
    if (e == hipSuccess) (void)hipEventRecord(e1, b->stream);
    std::vector<unsigned long long> landed(1 + (size_t)n * kLandedSlots);
    if (e == hipSuccess) {
        e = hipMemcpyAsync(landed.data(), b->d_cursor, sizeof(unsigned long long) * landed.size(),
                           hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        what = "irs_batch_run";
    }
    float ms = 0.0f;
    if (e == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) return hip_fail(e, what);
    for (irs_plan_s *p : b->plans) {        // a replay leaves no band the host knows of
        p->coef_c0 = -1;
        p->coef_c1 = -2;
    }
    if (stats) {
        for (int m = 0; m < n; ++m) {
            const irs_plan_s *p = b->plans[m];
            irs_map_stats &s = stats[m];
            std::memset(&s, 0, sizeof s);
            s.rays_shot = p->dg.nx * p->dg.ny;
            unsigned long long lm = 0;
            for (int k = 0; k < kLandedSlots; ++k) lm += landed[1 + (size_t)m * kLandedSlots + k];
            s.rays_landed = (int64_t)lm;
            s.rays_off = s.rays_shot - s.rays_landed;
            s.n_lens = p->n_lens;
            s.kappa_star_eff = p->kappa_star_eff;
            s.ms_total = ms;                      // the whole batch's graph launch
            if (p->params.method == IRS_DIRECT) s.direct_pairs = s.rays_shot * p->n_lens;
            s.super_cells = p->super_k;
            s.mid_cells = p->super_k > 0 ? p->mid_k : 0;
        }
    }
    set_error("");
    return IRS_OK;
}

irs_status irs_batch_get_info(irs_batch_t b, irs_batch_info *out)
{
    if (!b || !out) {
        set_error("irs_batch_get_info: NULL argument");
        return IRS_E_INVALID;
    }
    out->n_maps = (int32_t)b->plans.size();
    out->method = b->method;
    out->precision = b->precision;
    out->direct_variant = b->variant;
    out->blocks_per_cu = b->bpc;
    out->band_rows = b->band_rows;
    out->tuned = b->tuned ? 1 : 0;
    out->from_cache = b->from_cache ? 1 : 0;
    int64_t items = 0;
    for (const irs_plan_s *p : b->plans) items += direct_items(p, b->variant);
    out->work_items = b->method == IRS_DIRECT ? items : 0;
    out->tune_ms = b->tune_ms;
    out->whole_maps = b->whole ? 1 : 0;
    out->maps_per_launch = b->whole ? (int32_t)b->plans.size() : 0;
    return IRS_OK;
}

void irs_batch_free(irs_batch_t b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    dev_free(b->d_maps);
    dev_free(b->d_item_start);
    dev_free(b->d_cursor);
    dev_free(b->d_l3);
    dev_free(b->d_l3start);
    dev_free(b->d_l3cstart);
    for (hipStream_t ls : b->lanes) {
        (void)hipStreamSynchronize(ls);
        (void)hipStreamDestroy(ls);
    }
    for (hipEvent_t le : b->lane_done) (void)hipEventDestroy(le);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // extern "C"
