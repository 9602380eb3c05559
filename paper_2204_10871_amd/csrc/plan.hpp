// Internal plan object and the launch wrappers of the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/irs.h"
#include "device_common.hpp"
#include "geometry.hpp"

// Arguments of the direct-sum tile routines (one map).
namespace irs {
// A half-open range [a, b) of ray columns or rows: one tile of the level-3
// launch along that axis.
struct TileSpan {
    int32_t a, b;
};

struct DirectArgs {
    DevGeom g;
    const double *lx, *ly, *lm;          // sorted lenses (lm null: unit masses)
    const int32_t *cell_start;
    int32_t nl;
    int32_t pad_;
    int64_t ntx, ty0;                    // tiles per row; first tile row (queue kernels)
    int64_t row0, row1;                  // ray rows computed
    int64_t ray_first, ray_last;         // ray index range computed
    double *a1o, *a2o;                   // per-ray outputs (indexed r - ray_first) or
    int64_t *pixo;                       //   ... null
    uint32_t *counts;                    // map counts (null: per-ray outputs)
    unsigned long long *landed;          // rays binned
};
}  // namespace irs

struct irs_plan_s {
    irs_params params;
    irs::HostGeometry geo;
    irs::DevGeom dg;
    hipStream_t stream = nullptr;
    int device = 0;
    int64_t n_lens = 0;
    bool unit_mass = true;
    double kappa_star_eff = 0.0;
    int direct_variant = 1;              // FP32 direct tile shape (see k_direct.hip)
    bool no_alloc = false;               // set during irs_shoot_rows_noalloc: every
                                         // allocation site fails instead of allocating
    int64_t coef_budget = (int64_t)2 << 30;   // bytes for one band of level-2 coefficients

    // Lenses packed into level-1 cells (row-major cell order; inside a cell in
    // increasing input order).  FP64 positions and masses.
    double *d_x = nullptr, *d_y = nullptr, *d_m = nullptr;   // d_m null when unit masses
    int32_t *d_cell_start = nullptr;                         // n1x*n1y + 1
    uint32_t *d_cxy = nullptr;                               // per sorted lens: cy << 16 | cx
    int32_t *d_order = nullptr;                              // per sorted lens: input index
    double *d_xy = nullptr;                                  // (x, y) pairs, sorted order
    std::vector<int32_t> h_cell_start;                       // host copy (work counts)
    std::vector<int64_t> h_cell_cols;                        // ray columns per cell column

    // Level-2 coefficients of one band of level-1 rows: 10 doubles per point
    // (Re/Im of C0..C4), point (gx, gy) at ((gy - band_row0*q) * n1x*q + gx).
    int32_t super_k = 0;                  // super-cell side (cells), chosen once per plan
    int32_t mid_k = 0;                    // mid-cell side (cells), 0: no mid level
    double *d_mid = nullptr;              // mid-cell expansions (all rows), like d_super
    std::vector<char> mid_ok;
    void *d_rows = nullptr;               // level-3 row table (ny entries of 32 B)
    void *d_cols = nullptr;               // level-3 column table (nx entries of 48 B)
    // level-3 tiles: column tiles of <= 64 ray columns, row tiles of <= 32 ray
    // rows, following the level-1 cells where cells are wide (tall) enough
    irs::TileSpan *d_tcol = nullptr, *d_trow = nullptr;
    std::vector<irs::TileSpan> h_tcol, h_trow;
    double *d_coef = nullptr;
    int64_t coef_rows_cap = 0;   // level-1 rows the buffer holds
    int64_t coef_c0 = -1, coef_c1 = -2;   // level-1 rows whose coefficients it holds now
    double *d_part = nullptr;             // per-cell expansions (or per-chunk partials)
    size_t part_bytes = 0;
    int ring_fit = -1;                    // level-2 points may stage ring lenses (-1: unknown)
    // Two-level distant field: expansions of the super cells, kept while the
    // plan lives (its lenses never change); super_ok[Y]: row Y is computed.
    double *d_super = nullptr;
    std::vector<char> super_ok;
    double *d_super_part = nullptr;       // per-(super cell, lens chunk) partials
    size_t super_part_bytes = 0;

    // Learned interpolant (IRS_LEARNED): network, validation decision and the
    // corner table of one band of level-1 rows (4 doubles per corner:
    // Re A, Im A, Re A', Im A'; (qc + 1)^2 corners per cell).
    int learn_qc = 0;                     // squares per cell side; 0: no network
    bool learn_ok = false;                // validated; false: grid fallback
    float *d_theta = nullptr;             // FP32 parameters
    float *d_freqs = nullptr;             // 64 x 2
    void *d_wfwd = nullptr;               // BF16 forward fragments
    float *d_ltab = nullptr;              // the weights at the table's nodes (16 x nodes)
    void *d_lcol = nullptr;               // per ray column: square column, level-1 column
    int32_t lcol_qc = 0;                  // ... for this coarse grid
    double *d_corner = nullptr;
    int64_t corner_rows_cap = 0;
    int64_t corner_c0 = -1, corner_c1 = -2;

    // Scratch for host-side outputs.
    uint32_t *d_counts = nullptr;  // npix^2, used when counts are on the host
    unsigned long long *d_landed = nullptr;   // rays binned by the current call
    void *d_tmp = nullptr;
    size_t tmp_bytes = 0;
};

namespace irs {

// Two timing events, released on every path (create() may fail part-way).
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t create()
    {
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        return e;
    }
    EventPair() = default;
    EventPair(const EventPair &) = delete;
    EventPair &operator=(const EventPair &) = delete;
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Every device allocation of the library: hipMalloc, or hipErrorOutOfMemory
// (nothing allocated, *ptr null) for the allocation that the countdown of
// irs_debug_fail_alloc selects; and its release (NULL ignored).  Both keep
// the ledger of live allocations that irs_debug_live_allocs reports.
hipError_t dev_alloc_bytes(void **ptr, size_t bytes);
void dev_free(void *ptr);
template <class T>
inline hipError_t dev_alloc(T **ptr, size_t bytes)
{
    return dev_alloc_bytes((void **)ptr, bytes);
}

// Status plumbing shared by the launch wrappers and the C ABI.
void set_error(const std::string &msg);
irs_status hip_fail(hipError_t e, const char *what);

// Called where a plan buffer would be (re)allocated: the error of a call that
// must not allocate (p->no_alloc), else IRS_OK.
irs_status alloc_allowed(const irs_plan_s *p, const char *what);

#define IRS_HIP(call)                                                  \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return ::irs::hip_fail(e_, #call);       \
    } while (0)

// Level-1 packing: fills plan->d_x/d_y/d_m/d_cell_start from host lenses.
irs_status pack_level1(irs_plan_s *p, const double *hx, const double *hy, const double *hm);

// Per-call ray selection for the ray kernels: rays (i, j) with rows
// [row0, row1) and, when ray_first/ray_last are set, ray index r = j*nx + i
// in [ray_first, ray_last).  Outputs: per-ray arrays indexed r - ray_first
// (any may be null), or counts (null when per-ray outputs are wanted).
// Work and (optionally) HIP-event timings accumulated over one API call.
struct CallStats {
    int64_t level2_points = 0, level2_pairs = 0, direct_pairs = 0;
    double level2_flops = 0.0, level2_expand_flops = 0.0, ray_flops = 0.0;
    int32_t n_level2 = 0, n_rays = 0;
    double ms_level2 = 0.0, ms_level2_expand = 0.0, ms_rays = 0.0;
    bool timed = false;
    std::vector<hipEvent_t> ev;       // start/stop pairs, in launch order
    std::vector<int> ev_kind;         // 0 = level-2 expansion, 2 = level-2 points, 1 = rays
    // Record the start event of a launch of kind k (no-op unless timed).
    irs_status begin(hipStream_t s, int k);
    irs_status end(hipStream_t s);
    // Wait for the recorded events and sum their durations.
    irs_status collect();
    ~CallStats();
};

struct RaySel {
    CallStats *stats;
    int64_t row0, row1;
    int64_t ray_first, ray_last;
    double *alpha1, *alpha2;
    int64_t *pixel;
    uint32_t *counts;
    unsigned long long *landed;   // device counter of rays binned (with counts)
};

irs_status launch_direct(irs_plan_s *p, const RaySel &sel);
irs_status launch_interp(irs_plan_s *p, const RaySel &sel);
irs_status launch_learned(irs_plan_s *p, const RaySel &sel);
void learn_release(irs_plan_s *p);

// FP32 direct tile shapes: rays per lane x lenses per LDS stage.
constexpr int kDirectVariants = 3;
int direct_variant_rows(int v);          // ray rows per tile of shape v
const char *direct_variant_name(int v);

// Batched direct sums: one persistent launch over every map's tiles.
// maps: device table; item_start: device prefix of tiles per map; cursor:
// device counter, zero before the launch.  blocks: persistent grid size.
irs_status launch_direct_queue(hipStream_t s, int precision, bool unit, int variant,
                               const DirectArgs *maps, const int64_t *item_start,
                               int32_t nmaps, unsigned long long *cursor, int blocks);
// Tiles (FP32) or 256-ray groups (FP64) of a whole map, and its DirectArgs.
int64_t direct_items(const irs_plan_s *p, int variant);
DirectArgs direct_args_full(const irs_plan_s *p, int variant, uint32_t *counts,
                            unsigned long long *landed);
// Level-2 buffers sized for whole-map bands, allocated now (before a capture).
irs_status interp_prepare(irs_plan_s *p);
// Bytes per level-1 row of the level-2 coefficient band and of the cell
// expansions (0 when the plan has none).
void interp_band_row_bytes(const irs_plan_s *p, int64_t &coef_row, int64_t &part_row);
// IRS_OK if a call of the interpolated method on rows of this plan would
// allocate nothing but its coefficient band and cell expansions: the row
// table, the super- and mid-cell expansions and their partials exist at
// whole-map size.  Otherwise an error with a message.
irs_status interp_tables_ready(irs_plan_s *p);
// Interpolated batches with every map's level 2 resident at once: the bytes
// a map's whole-map level-2 buffers take; allocate them (before a capture);
// compute a map's whole level-2 field on its stream; a map's level-3 launch
// arguments (interp_map_args_bytes() bytes into out); the device table of n
// maps' arguments (args, in launch order) and their tile and corner-block
// prefixes (d_maps: n args, d_start and d_cstart: n + 1 each; copied and
// synchronised on s); and the level 3 of those maps as one launch over every
// map's tiles (a workgroup a tile) plus one over their corner-cell rays.
int64_t interp_whole_map_bytes(const irs_plan_s *p);
irs_status interp_prepare_whole(irs_plan_s *p);
irs_status interp_level2_whole(irs_plan_s *p);
size_t interp_map_args_bytes();
irs_status interp_map_args(irs_plan_s *p, uint32_t *counts, unsigned long long *landed,
                           void *out);
irs_status interp_maps_table(const void *args, int32_t n, void *d_maps, int64_t *d_start,
                             int64_t *d_cstart, hipStream_t s);
irs_status launch_interp_maps(hipStream_t s, bool unit, const void *args, const void *d_maps,
                              const int64_t *d_start, const int64_t *d_cstart, int32_t n);
// Fill kernel (graph-safe zeroing): n 32-bit words.
irs_status launch_zero(hipStream_t s, void *ptr, size_t n_words);

}  // namespace irs
