/*
 * irs.h -- C ABI of the MI355X (gfx950) inverse-ray-shooting library.
 *
 * The library computes gravitational-microlensing magnification maps by the
 * inverse ray-shooting method of Zheng et al., "An Improved GPU-Based
 * Ray-Shooting Code for Gravitational Microlensing" (arXiv 2204.10871):
 *
 *   1. deflection of every image-plane ray by N_* point masses, a smooth
 *      convergence kappa_s and an external shear gamma, on the rectangular
 *      lens plane with its negative mass sheet (Eq. 6 and Appendix A);
 *   2. optionally the three-level-grid interpolation: lenses packed into
 *      level-1 cells, distant lenses and the sheet summed with Taylor
 *      coefficients up to fourth order at level-2 points, nearby lenses summed
 *      exactly for every level-3 ray (Sec. 2.4 and its flow chart);
 *   3. binning of the mapped rays beta = theta - alpha (Eq. 4) into
 *      source-plane pixel counts N_ij, with Mag_ij = N_ij S_I / S_S
 *      (flow chart, "Calculate the magnification of each pixel").
 *
 * Conventions shared by every entry point
 *   - Angles are in units of the Einstein angle of the mean lens mass (Eq. 3);
 *     masses are in units of that mean mass.
 *   - Geometry: protective border P = 10 sqrt(kappa_*), lens/image rectangle
 *     I_x = (S+2P)/|1-kappa-gamma|, I_y = (S+2P)/|1-kappa+gamma| centred on the
 *     origin (flow chart, "Calculate the size of the Protective Border").
 *   - Rays form a regular nx x ny grid over the rectangle, spacing
 *     dx3 = sqrt(I_x I_y / N_rays) rounded to whole rows/columns, each ray at
 *     its grid cell's centre.  Ray r = j*nx + i (row-major, i along theta_1).
 *   - The source map covers [-S/2, S/2)^2 with npix_side^2 pixels; pixel index
 *     p = iy*npix_side + ix with ix = floor((beta_1 + S/2)/(S/npix_side));
 *     rays outside the map are not counted (index -1 where reported).
 *   - Status codes are returned; nothing throws across the ABI.  On error no
 *     output buffer is partially written unless stated, and irs_last_error()
 *     returns a message for the calling thread.
 *   - Host pointers unless IRS_OUT_ON_DEVICE is passed in a call's flags, in
 *     which case output pointers are device pointers on the plan's device.
 *   - A plan is not reentrant: calls on one plan must not overlap.  Distinct
 *     plans may be used concurrently on distinct streams.
 */
#ifndef IRS_H
#define IRS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct irs_plan_s *irs_plan_t;     /* opaque, owned by the library */

typedef enum {
    IRS_OK = 0,
    IRS_E_INVALID = 1,      /* an argument is out of range or NULL            */
    IRS_E_CRITICAL = 2,     /* |1-kappa-gamma| or |1-kappa+gamma| < crit_eps:  */
                            /* the shooting rectangle is unbounded            */
    IRS_E_NOMEM = 3,        /* a device allocation failed                     */
    IRS_E_DEVICE = 4,       /* a HIP runtime call or kernel launch failed     */
    IRS_E_UNSUPPORTED = 5   /* method / precision combination not provided    */
} irs_status;

/* irs_params.method */
enum { IRS_DIRECT = 0,      /* sum over every lens for every ray (Eq. 6)       */
       IRS_INTERP = 1,      /* three-level-grid interpolation (Sec. 2.4)       */
       IRS_LEARNED = 2 };   /* Sec. 2.4's split with a learned interpolant of the
                               distant field on a coarse grid (see irs_learn)  */

/* irs_params.precision */
enum { IRS_FP64 = 0,        /* every step in double precision                  */
       IRS_FP32_KAHAN = 1 };/* direct sum in FP32 with tile-local coordinates
                               and compensated accumulation; FP64 for the macro
                               term, the sheet, the near-lens residuals and the
                               level-2 coefficients                            */

/* irs_params.flags */
#define IRS_SHEET_OFF      (1ull << 0)  /* omit the negative mass sheet (point-lens tests) */
#define IRS_LEVEL2_PAPER   (1ull << 1)  /* level-2 coefficients by direct summation of the
                                           distant lenses at every level-2 point, as in
                                           the paper, instead of through one local
                                           expansion per level-1 cell (same values to
                                           FP64 rounding; kept for comparison)          */
#define IRS_CIRCLE         (1ull << 2)  /* circular lens plane (Sec. 2.1): the lenses fill
                                           the image rectangle's circumscribed circle,
                                           radius R = sqrt(I_x^2 + I_y^2)/2, and the
                                           negative sheet deflects by -kappa_* theta
                                           (Eq. 9) instead of the rectangle's Appendix A
                                           forms; n_stars_expected = round(kappa_* R^2).
                                           The caller's lenses should lie in the circle.
                                           Direct method in FP64 only (otherwise
                                           IRS_E_UNSUPPORTED from irs_geometry/irs_plan) */
/* per-call flags */
#define IRS_OUT_ON_DEVICE  (1ull << 8)  /* output pointers are device pointers          */
#define IRS_TIME_PHASES    (1ull << 9)  /* time each kernel launch with HIP events on
                                           the plan's stream (fills the ms_* stats)     */

typedef struct {
    double   kappa_star;          /* compact convergence kappa_* (Eq. 2), >= 0        */
    double   kappa_c;             /* smooth convergence kappa_s (Eq. 2), >= 0         */
    double   gamma;               /* external shear                                   */
    double   source_side;         /* S_scale, side of the source map, > 0             */
    int64_t  npix_side;           /* pixels per side; N_pix = npix_side^2, <= 46340   */
    double   rays_per_pixel;      /* N_av; used when n_rays <= 0                      */
    int64_t  n_rays;              /* > 0: total ray count instead of N_av * N_pix     */
    double   border;              /* < 0: P = 10 sqrt(kappa_*); >= 0: explicit P      */
    int32_t  method;              /* IRS_DIRECT, IRS_INTERP or IRS_LEARNED             */
    int32_t  precision;           /* IRS_FP64 or IRS_FP32_KAHAN                        */
    double   level2_spacing;      /* > 0: explicit level-2 spacing dx2                */
    double   level2_ray_multiple; /* > 0: dx2 = this many ray spacings; both <= 0:   */
                                  /* dx2 = dx1/20 (flow chart, level-2 resolution)   */
    double   crit_eps;            /* <= 0: 1e-3                                        */
    uint64_t flags;               /* IRS_SHEET_OFF, IRS_LEVEL2_PAPER, IRS_CIRCLE       */
} irs_params;

typedef struct {
    double  kappa;                /* kappa_* + kappa_s                                */
    double  border;               /* protective border P                              */
    double  ix, iy;               /* rectangle sides I_x, I_y                          */
    double  a1, a2, b1, b2;       /* rectangle [a1,a2] x [b1,b2]                       */
    int64_t n_rays_target;        /* N_av * N_pix or n_rays                            */
    double  dx3;                  /* sqrt(I_x I_y / N_rays)                            */
    int64_t nx, ny;               /* ray grid                                          */
    double  ray_dx, ray_dy;       /* I_x/nx, I_y/ny                                    */
    int64_t n_lens;               /* lens count the level-1 grid was sized for         */
    double  dx1;                  /* min(L0, min(I_x, I_y)/10), L0 = sqrt(I_x I_y/N_*) */
    int64_t n1x, n1y;             /* level-1 cells tiling the rectangle (<= dx1 side)   */
    double  dx2;                  /* requested level-2 spacing                         */
    int64_t q;                    /* level-2 points per level-1 cell side, round(dx1/dx2) */
    double  dpix;                 /* S / npix_side                                     */
    double  s_img, s_src;         /* S_I = ray_dx * ray_dy, S_S = dpix^2               */
    double  mu_th;                /* 1/((1-kappa)^2 - gamma^2)                          */
    int64_t n_stars_expected;     /* round(kappa_* I_x I_y / pi); IRS_CIRCLE:
                                     round(kappa_* lens_radius^2)                    */
    double  lens_radius;          /* IRS_CIRCLE: sqrt(I_x^2 + I_y^2)/2; else 0        */
} irs_geometry_info;

typedef struct {
    int64_t rays_shot;            /* rays evaluated by the call                       */
    int64_t rays_landed;          /* rays counted into the map                        */
    int64_t rays_off;             /* rays that left the map                           */
    int64_t n_lens;               /* lenses in the plan                               */
    double  kappa_star_eff;       /* pi * sum(m) / (I_x I_y)                          */
    double  ms_total;             /* wall time of the call on the plan's stream       */
    /* work done by the call (interpolation: level-2 points computed and
       (point, distant lens) pairs summed; direct: ray-lens pairs)                   */
    int64_t level2_points;
    int64_t level2_pairs;         /* (point, distant lens) pairs the paper's form sums */
    int64_t direct_pairs;
    double  level2_flops;         /* algorithmic flops of the level-2 kernels used     */
    double  level2_expand_flops;  /* ... of which the per-cell expansion kernel        */
    /* with IRS_TIME_PHASES: summed HIP-event durations of the launches          */
    int32_t n_level2_launches;    /* level-2 (far field) launches                     */
    int32_t n_ray_launches;       /* level-3 or direct-sum launches                   */
    double  ms_level2;            /* all level-2 launches                             */
    double  ms_level2_expand;     /* the per-cell expansion (or per-point sum) kernel  */
    double  ms_rays;
    int32_t learned;              /* IRS_LEARNED plans: 1 if the network was used,    */
                                  /* 0 if the grid-interpolation fallback was          */
    int32_t pad_;
    double  ray_flops;            /* algorithmic FP64 flops of the level-3 launches   */
                                  /* (interpolation; 46 per ray + 10 per near lens)   */
    int32_t super_cells;          /* sides, in level-1 cells, of the super and mid     */
    int32_t mid_cells;            /* cells of the distant-field tree the plan uses     */
                                  /* (0: level absent or not built yet)                */
} irs_map_stats;

/*
 * irs_geometry -- derive the plan geometry from the inputs, on the host.
 * Follows the flow chart of Sec. 2.4 (border, rectangle, level-1/2/3
 * resolutions, pixel areas).  n_lens sizes the level-1 grid (0 allowed).
 * Needs no GPU.  Errors: IRS_E_INVALID (NULL or out-of-range input),
 * IRS_E_CRITICAL (near a critical line).
 */
irs_status irs_geometry(const irs_params *params, int64_t n_lens, irs_geometry_info *out);

/*
 * irs_level1_span -- the rays of level-1 row or column c of a geometry: for
 * axis 1 the ray rows [*first, *last), for axis 0 the ray columns, whose
 * level-2 points lie in that level-1 row (column).  Ray row j lies in level-2
 * row floor((2j+1) n1y q / (2 ny)) (the level-2 points are the centres of a
 * q x q split of every level-1 cell, Sec. 2.4 flow chart).  Host only.
 * Errors: IRS_E_INVALID (NULL, axis not 0/1, c outside the level-1 grid).
 */
irs_status irs_level1_span(const irs_geometry_info *geo, int32_t axis, int64_t c,
                           int64_t *first, int64_t *last);

/*
 * irs_source_side -- the source side S for which the rectangle of params
 * holds n_star lenses by the lens-count rule round(kappa_* I_x I_y / pi)
 * (lens density kappa_* / pi at unit mean mass, Appendix A's sheet density;
 * I_x, I_y from the protective border and S, Sec. 2.3): the smallest S, to
 * bisection precision, whose n_stars_expected is >= n_star.  params'
 * source_side, npix_side and ray counts are ignored.  Host only.
 * Errors: IRS_E_INVALID, IRS_E_CRITICAL.
 */
irs_status irs_source_side(const irs_params *params, int64_t n_star, double *source_side);

/*
 * irs_plan -- create a plan: validate inputs, derive the geometry, copy the
 * lenses to the device and pack them into level-1 cells (flow chart, "Lenses
 * packed into level-1 grids").
 *   x, y : n_lens lens positions (host, FP64); m : masses or NULL for all 1.
 *          The arrays are copied; the caller keeps ownership.  IRS_INTERP
 *          and IRS_LEARNED plans need every lens inside the rectangle
 *          [a1, a2] x [b1, b2] (to 1e-6 of a level-1 cell): the distant
 *          field's series assume each lens inside its level-1 cell.
 *   hip_stream : hipStream_t to run on, or NULL for the default stream.
 *   out : receives the plan handle (NULL on error).
 * Errors: IRS_E_INVALID (NULL or out-of-range input, a lens position not
 * finite, a mass not finite or negative, a lens outside the rectangle of an
 * interpolated plan), IRS_E_CRITICAL, IRS_E_UNSUPPORTED, IRS_E_NOMEM,
 * IRS_E_DEVICE.  The call returns when the plan is ready.
 */
irs_status irs_plan(const irs_params *params, int64_t n_lens, const double *x,
                    const double *y, const double *m, void *hip_stream, irs_plan_t *out);

/*
 * irs_deflect_grid -- per-ray results for rays [first_ray, first_ray + n):
 * alpha (FP64, Eq. 6 evaluated by the plan's method and precision) and the
 * source pixel index (int64, -1 off the map).  Any output may be NULL.  The
 * per-ray arithmetic is exactly that of irs_shoot_rows / irs_shoot_map.
 * Errors: IRS_E_INVALID (range outside [0, nx*ny)), IRS_E_NOMEM, IRS_E_DEVICE.
 */
irs_status irs_deflect_grid(irs_plan_t plan, int64_t first_ray, int64_t n, double *alpha1,
                            double *alpha2, int64_t *pixel, uint64_t flags);

/*
 * irs_shoot_rows -- shoot ray rows [row0, row0 + nrows) and ADD their pixel
 * counts to `counts` (npix_side^2 uint32, row-major; host or device per
 * flags).  Disjoint row ranges add up exactly to the full map, so a long map
 * can be shot in bands and resumed.  stats may be NULL.
 * Errors: IRS_E_INVALID, IRS_E_NOMEM, IRS_E_DEVICE.
 */
irs_status irs_shoot_rows(irs_plan_t plan, int64_t row0, int64_t nrows, uint32_t *counts,
                          irs_map_stats *stats, uint64_t flags);

/*
 * irs_shoot_rows_noalloc -- irs_shoot_rows for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): rays of rows [row0, row0 + nrows) are shot and their
 * pixel counts ADDED to `counts`, a DEVICE pointer to npix_side^2 uint32 on
 * the plan's device, with the same kernels and results, bit for bit, as
 * irs_shoot_rows.  The call allocates nothing: its scratch -- the landed-ray
 * counters and, for IRS_INTERP plans, the level-2 coefficient band and cell
 * expansions -- lives in a static 64 MiB device array that each GPU holds
 * until the process ends; the counters are cleared by a fill kernel, not a
 * memset.  Every call on one GPU shares that array, so calls that overlap on
 * one GPU (other plans or threads included) race; serialise them.
 *   rays_landed : host int64 receiving the rays binned by the call, or NULL
 *                 (then the call only enqueues work on the plan's stream and
 *                 does not synchronise).
 * Requirements: the plan's device is the current device; IRS_DIRECT plans
 * need nothing else; IRS_INTERP plans need one level-1 row of level-2 scratch
 * (n1x q^2 80 bytes plus the cell expansions) to fit in the array, and the
 * plan's own tables (row table, super- and mid-cell expansions) allocated at
 * whole-map size, which one irs_shoot_map on the plan does.
 * Errors: IRS_E_INVALID (NULL, range, another device current, a level-1 row
 * needing more scratch than the array holds, tables not allocated; nothing
 * is launched then), IRS_E_UNSUPPORTED (IRS_LEARNED plans), IRS_E_DEVICE.
 */
irs_status irs_shoot_rows_noalloc(irs_plan_t plan, int64_t row0, int64_t nrows,
                                  uint32_t *counts, int64_t *rays_landed);

/*
 * irs_shoot_map -- shoot every ray and WRITE the pixel counts N_ij to
 * `counts` (npix_side^2 uint32).  Mag_ij = N_ij * s_img / s_src.
 * Errors: as irs_shoot_rows.
 */
irs_status irs_shoot_map(irs_plan_t plan, uint32_t *counts, irs_map_stats *stats,
                         uint64_t flags);

/*
 * irs_plan_set_direct_variant -- FP32 direct tile shape of the plan (0, 1, 2 as
 * in irs_batch_info.direct_variant; default 1).  Every shape gives the same
 * results bit for bit; only the speed differs.  IRS_E_INVALID if out of range.
 */
irs_status irs_plan_set_direct_variant(irs_plan_t plan, int32_t variant);

/* irs_plan_geometry -- the geometry the plan uses (n_lens = the plan's lens count). */
irs_status irs_plan_geometry(irs_plan_t plan, irs_geometry_info *out);

/*
 * irs_plan_level1 -- the plan's packing of the lenses into level-1 cells (Sec.
 * 2.4 flow chart, "Lenses packed into level-1 grids").  Host buffers owned by
 * the caller: cell_start[n1x n1y + 1], cell c = cy n1x + cx holding packed
 * lenses [cell_start[c], cell_start[c+1]); order[n_lens], order[k] = input
 * index of packed lens k.  Inside a cell the packed order is the input order
 * (the packing is a stable sort by cell).  order may be NULL when the plan has
 * no lenses.  IRS_E_INVALID on a NULL argument, IRS_E_HIP if the copy fails.
 */
irs_status irs_plan_level1(irs_plan_t plan, int32_t *cell_start, int32_t *order);

/* irs_free -- release a plan and all its device memory.  NULL is ignored. */
void irs_free(irs_plan_t plan);

/* irs_last_error -- message for the last failed call on this thread ("" if none). */
const char *irs_last_error(void);

/*
 * irs_debug_fail_alloc -- fault injection for tests of the out-of-memory
 * paths: the next `after` device allocations of the library (any thread, any
 * plan or batch, set-up included) succeed and the one after them fails as an
 * exhausted hipMalloc would (the call returns IRS_E_NOMEM); after < 0
 * switches it off.  Process-wide.  Returns IRS_OK.
 */
irs_status irs_debug_fail_alloc(int64_t after);

/*
 * irs_debug_live_allocs -- the library's device allocations that are live
 * now (made and not yet freed, over every plan and batch of the process):
 * their number into *count and their total size in bytes into *bytes.  For
 * leak checks that must not depend on what the HIP runtime itself keeps.
 * IRS_E_INVALID on a NULL argument.
 */
irs_status irs_debug_live_allocs(int64_t *count, int64_t *bytes);

/* ------------------------------------------------------------------------ */
/* Batches of independent maps.                                              */
/* ------------------------------------------------------------------------ */

typedef struct irs_batch_s *irs_batch_t;   /* opaque, owned by the library */

typedef struct {
    int32_t n_maps;
    int32_t method, precision;
    int32_t direct_variant;       /* FP32 direct tile shape: 0 = 4 rays/lane x 512 lenses
                                     per LDS stage, 1 = 8 x 256, 2 = 16 x 128          */
    int32_t blocks_per_cu;        /* persistent workgroups per compute unit (direct)  */
    int32_t band_rows;            /* level-1 rows per level-2 band (interpolation,     */
                                  /* 0: every map's whole level-2 field at once)        */
    int32_t tuned;                /* 1 if the settings came from the autotuner         */
    int32_t from_cache;           /* 1 if they were read from the tuning cache         */
    int64_t work_items;           /* queue items of the persistent launch (direct)     */
    double  tune_ms;              /* time the autotuner spent measuring                */
    int32_t whole_maps;           /* interpolation: 1 if every map's level-2 field is  */
                                  /* resident at once and level 3 runs as one launch   */
                                  /* over every map's tiles                            */
    int32_t maps_per_launch;      /* ... maps in that launch (the batch's n; 0 if not) */
} irs_batch_info;

/*
 * Environment: IRS_BATCH_BANDS set (to anything but "0") when a batch is
 * created keeps an interpolated batch band by band per map (no whole-map
 * level 2); IRS_TUNE_CACHE names the tuning cache (irs_batch_tune).
 *
 * irs_batch_create -- group n plans (the motivation: the many maps needed to
 * sample lens-model parameters, Sec. 4) into one batch.  All plans must share
 * method, precision and device, and for the direct method the mass kind
 * (unit or not).  The plans stay owned by the caller and must outlive the
 * batch; the batch runs them on its own stream (hip_stream, or a new one if
 * NULL).  Errors: IRS_E_INVALID, IRS_E_UNSUPPORTED, IRS_E_NOMEM, IRS_E_DEVICE.
 */
irs_status irs_batch_create(const irs_plan_t *plans, int32_t n, void *hip_stream,
                            irs_batch_t *out);

/*
 * irs_batch_tune -- choose the batch's launch settings by measurement on this
 * device: for the direct method the tile shape and the persistent grid size,
 * timed on the heaviest map's first tiles; for the interpolation, when the
 * maps' level-2 fields do not fit at once, the band height, timed on one band
 * of the heaviest map (when they fit, level 3 is one launch of a workgroup
 * per tile and nothing is measured).  cache_path (or, if NULL,
 * the IRS_TUNE_CACHE environment variable; neither: no cache) is a text file
 * of "key = settings" lines keyed by method, precision, mass kind, lens-count
 * and aspect buckets; a cached key is reused without measuring.  The chosen
 * tile shape is also set on every plan of the batch.
 */
irs_status irs_batch_tune(irs_batch_t batch, const char *cache_path);

/*
 * irs_batch_run -- every map of the batch in one graph launch: for the direct
 * method one persistent kernel drains a device queue of (map, ray tile)
 * items ordered longest map first; for the interpolation every map's level-2
 * field (on parallel branches of the graph), then level 3 as one launch of a
 * workgroup per tile over every map's tiles laid end to end, longest map
 * first, and one launch over every map's corner-cell rays -- when all maps' level-2 fields fit in device memory at once
 * (60% of the free memory at irs_batch_create, one mass kind); else the maps'
 * band launches on parallel branches.  counts[k] is a DEVICE pointer to map k's
 * npix_side^2 uint32 counts, overwritten.  The graph is captured on the first
 * call and replayed while the counts pointers stay the same.  stats: n entries
 * or NULL.  Results equal per-plan irs_shoot_map bit for bit.
 */
irs_status irs_batch_run(irs_batch_t batch, uint32_t *const *counts, irs_map_stats *stats,
                         uint64_t flags);

/* irs_batch_get_info -- the batch's current settings. */
irs_status irs_batch_get_info(irs_batch_t batch, irs_batch_info *out);

/* irs_batch_free -- release a batch (not its plans).  NULL is ignored. */
void irs_batch_free(irs_batch_t batch);

/* ------------------------------------------------------------------------ */
/* Learned interpolant of the distant-lens field (method IRS_LEARNED).       */
/* ------------------------------------------------------------------------ */
/*
 * The interpolation of Sec. 2.4 sums the nearby lenses (3 x 3 level-1 cells)
 * exactly and takes the distant lenses and the sheet from a fourth-order
 * Taylor series about the ray's level-2 point.  IRS_LEARNED keeps that split
 * and replaces the Taylor series by a learned interpolant on a coarser grid.
 * Every level-1 cell is cut into coarse x coarse squares; at their corners the
 * plan computes, in FP64, the cell's distant field A(z) (distant lenses plus
 * the analytic part of the sheet, outside the four corner cells) and A'(z).
 * For a ray at z in a square with corners z_c, offset h in [0,1]^2:
 *   I(z)  = sum_c w_c(h) (A_c + A'_c (z - z_c))       bilinear weights w_c,
 *   D     = (delta_c, eps_c) / sigma, delta_c = (A'_c - mean A') s,
 *           eps_c = A_c - mean A - mean A' (z_c - mean z_c), s = mean side,
 *           sigma = max |delta_c|, |eps_c|,
 *   A(z) ~= I(z) + sigma sum_k L_k(h) D_k,   k = 0..7,
 * with L(h) in C^8 from a Fourier-feature MLP: features sin and cos of
 * 2 pi f_j . (h - 1/2) for 64 frequencies f_j, four hidden ReLU layers of 128,
 * 16 outputs (L_k = y_2k + i y_2k+1).  Weights and activations are BF16 on the
 * matrix cores with FP32 accumulation.  The network is trained on the GPU
 * (Adam, FP32 master weights) on exact samples of A that the plan computes,
 * then validated on samples from other rows; if it misses the tolerance the
 * plan shoots with the grid interpolation of IRS_INTERP instead (fallback).
 * The paper has no learned part; this is the library's extension of Sec. 2.4.
 *
 * Parameter vector: IRS_LEARN_NPARAMS FP32 numbers W1 (128 x 128, row-major,
 * row = output unit), b1 (128), W2, b2, W3, b3, W4, b4, W5 (16 x 128), b5 (16).
 * Frequencies: IRS_LEARN_NFREQ x 2 FP32, row j = (f_jx, f_jy).
 */
#define IRS_LEARN_NFREQ    64
#define IRS_LEARN_NPARAMS  68112
#define IRS_LEARN_FIELDS   24   /* floats per sample record (irs_learn_samples) */

typedef struct {
    int32_t  coarse;        /* squares per level-1 cell side, 1..32              */
    int32_t  train_rows;    /* level-1 rows the training samples come from,      */
                            /* spread evenly over the map                        */
    int64_t  n_samples;     /* training samples                                  */
    int64_t  n_val;         /* validation samples, from rows between those       */
    int32_t  batch;         /* samples per Adam step, multiple of 256            */
    int32_t  steps;         /* Adam steps                                         */
    float    lr, lr_final;  /* learning rate, cosine decay from lr to lr_final    */
    float    beta1, beta2, adam_eps;
    int32_t  pad_;
    uint64_t seed;          /* sample positions and initial weights               */
    double   tol_mean;      /* fallback if validation mean |error| exceeds this;  */
                            /* <= 0: 2.5e-5 dpix                                  */
    double   tol_p9999;     /* ... or its 99.99th percentile; <= 0: 2.5e-3 dpix   */
} irs_learn_params;

typedef struct {
    int64_t n_samples, n_val, steps;
    double  loss_first, loss_last;      /* mean training loss of the first and last
                                           5% of the steps (normalised units)    */
    double  val_mean_abs, val_p9999_abs, val_max_abs;    /* |learned - A|, theta_E */
    double  base_mean_abs, base_p9999_abs, base_max_abs; /* |I - A|: same grid,
                                                            no network            */
    double  tol_mean, tol_p9999;
    int32_t fallback;       /* 1: tolerance missed; the plan uses grid interpolation */
    int32_t coarse;
    double  ms_samples, ms_train, ms_validate;
    int64_t corner_bytes_per_row;       /* learned table per level-1 row          */
    int64_t coef_bytes_per_row;         /* grid-interpolation table per row       */
} irs_learn_report;

/* irs_learn_defaults -- default training settings (coarse 16, 2e6 samples over 8
   rows, 2e5 validation samples, batch 8192, 6000 steps, lr 2e-3 -> 2e-5). */
irs_status irs_learn_defaults(irs_learn_params *out);

/*
 * irs_learn -- generate exact samples, train the network and validate it on an
 * IRS_LEARNED plan.  freqs: IRS_LEARN_NFREQ x 2 host floats; theta0: initial
 * parameters (host, IRS_LEARN_NPARAMS) or NULL for a seeded He initialisation.
 * report may be NULL.  The trained network is tabulated over the in-square
 * offset (irs_learn_weights) and the validation measures the tabulated
 * weights, which the rays use.  Afterwards the plan's shooting calls use
 * them, or the grid interpolation if report->fallback is 1.
 * Errors: IRS_E_INVALID (not an IRS_LEARNED plan, settings out of range),
 * IRS_E_UNSUPPORTED (IRS_LEVEL2_PAPER plans), IRS_E_NOMEM, IRS_E_DEVICE.
 */
irs_status irs_learn(irs_plan_t plan, const irs_learn_params *lp, const float *freqs,
                     const float *theta0, irs_learn_report *report);

/*
 * irs_learn_set -- install a network (for example one saved with irs_learn_get)
 * on an IRS_LEARNED plan, validate it as irs_learn does (lp: NULL for the
 * defaults; only coarse, n_val, train_rows, seed and the tolerances are read)
 * and decide the fallback.  Host arrays as for irs_learn.
 */
irs_status irs_learn_set(irs_plan_t plan, const irs_learn_params *lp, const float *freqs,
                         const float *theta, irs_learn_report *report);

/* irs_learn_get -- the plan's network: frequencies, parameters (host) and coarse.
   IRS_E_INVALID if the plan has none. */
irs_status irs_learn_get(irs_plan_t plan, float *freqs, float *theta, int32_t *coarse);

/*
 * irs_learn_corners -- the corner table of level-1 rows [row0, row0 + nrows):
 * out (host, FP64) [((r - row0) n1x + cx) (coarse+1)^2 + b (coarse+1) + a] x 4
 * = Re A, Im A, Re A', Im A' at corner (a, b) of cell (cx, r), corner position
 * (a1 + (cx coarse + a) sx, b1 + (r coarse + b) sy), sx = I_x/(n1x coarse),
 * sy = I_y/(n1y coarse).  For checking the learned path.
 */
irs_status irs_learn_corners(irs_plan_t plan, int32_t coarse, int64_t row0, int64_t nrows,
                             double *out);

/*
 * irs_learn_samples -- the exact samples irs_learn trains on: per_cell samples
 * in every cell of level-1 rows [row0, row0 + nrows), positions from a
 * counter-based generator (seed, sample index).  out: DEVICE floats, field f of
 * sample k at out[f n + k], n = nrows n1x per_cell; fields 0-1 h, 2-17 D
 * (Re, Im of D_0..D_7), 18-19 T = (A - I)/sigma, 20 sigma, 21 cx, 22 cy,
 * 23 square b coarse + a.
 */
irs_status irs_learn_samples(irs_plan_t plan, int32_t coarse, int64_t row0, int64_t nrows,
                             int32_t per_cell, uint64_t seed, float *out);

/*
 * irs_learn_weights -- the plan's learned weights L(h) at n in-square offsets,
 * exactly as its rays take them: the network's 16 outputs at the 33 x 33
 * nodes (a/32, b/32) of the unit square, tabulated whenever irs_learn or
 * irs_learn_set validates a network, blended bilinearly between the four
 * nodes around h (h clamped to [0, 1]^2).  h: DEVICE, 2 x n (hx row then hy
 * row); y: DEVICE, 16 x n (y[o n + k]).  Runs on the plan's stream and waits
 * for it.  IRS_E_INVALID on a NULL argument, n < 0 or a plan with no network.
 */
irs_status irs_learn_weights(irs_plan_t plan, int64_t n, const float *h, float *y);

/*
 * irs_mlp_forward -- the network's outputs y (DEVICE, 16 x n: y[o n + k]) at
 * offsets h (DEVICE, 2 x n: hx row then hy row), with the inference kernel.
 * freqs, theta: host arrays as above.  hip_stream: NULL for the default stream.
 */
irs_status irs_mlp_forward(int64_t n, const float *freqs, const float *theta,
                           const float *h, float *y, void *hip_stream);

/*
 * irs_mlp_loss_grad -- training loss (1/n) sum |sum_k L_k D_k - T|^2 over the n
 * sample records (DEVICE, IRS_LEARN_FIELDS x n as irs_learn_samples writes)
 * and its gradient (host, IRS_LEARN_NPARAMS floats) from the training kernels.
 */
irs_status irs_mlp_loss_grad(int64_t n, const float *freqs, const float *theta,
                             const float *samples, double *loss, float *grad,
                             void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* IRS_H */
