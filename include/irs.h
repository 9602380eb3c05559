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
 *      exactly for every level-3 ray (Sec. 2.3 and the flow chart of Sec. 2.4);
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
       IRS_INTERP = 1 };    /* three-level-grid interpolation (Sec. 2.3)       */

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
    int32_t  method;              /* IRS_DIRECT or IRS_INTERP                          */
    int32_t  precision;           /* IRS_FP64 or IRS_FP32_KAHAN                        */
    double   level2_spacing;      /* > 0: explicit level-2 spacing dx2                */
    double   level2_ray_multiple; /* > 0: dx2 = this many ray spacings; both <= 0:   */
                                  /* dx2 = dx1/20 (flow chart, level-2 resolution)   */
    double   crit_eps;            /* <= 0: 1e-3                                        */
    uint64_t flags;               /* IRS_SHEET_OFF, IRS_LEVEL2_PAPER                   */
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
    int64_t n_stars_expected;     /* round(kappa_* I_x I_y / pi)                       */
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
 * irs_plan -- create a plan: validate inputs, derive the geometry, copy the
 * lenses to the device and pack them into level-1 cells (flow chart, "Lenses
 * packed into level-1 grids").
 *   x, y : n_lens lens positions (host, FP64); m : masses or NULL for all 1.
 *          The arrays are copied; the caller keeps ownership.
 *   hip_stream : hipStream_t to run on, or NULL for the default stream.
 *   out : receives the plan handle (NULL on error).
 * Errors: IRS_E_INVALID, IRS_E_CRITICAL, IRS_E_UNSUPPORTED, IRS_E_NOMEM,
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

/* irs_free -- release a plan and all its device memory.  NULL is ignored. */
void irs_free(irs_plan_t plan);

/* irs_last_error -- message for the last failed call on this thread ("" if none). */
const char *irs_last_error(void);

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
    int32_t band_rows;            /* level-1 rows per level-2 band (interpolation)    */
    int32_t tuned;                /* 1 if the settings came from the autotuner         */
    int32_t from_cache;           /* 1 if they were read from the tuning cache         */
    int64_t work_items;           /* queue items of the persistent launch (direct)     */
    double  tune_ms;              /* time the autotuner spent measuring                */
} irs_batch_info;

/*
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
 * timed on the heaviest map's first tiles; for the interpolation the band
 * height, timed on one band of the heaviest map.  cache_path (or, if NULL,
 * the IRS_TUNE_CACHE environment variable; neither: no cache) is a text file
 * of "key = settings" lines keyed by method, precision, mass kind, lens-count
 * and aspect buckets; a cached key is reused without measuring.  The chosen
 * tile shape is also set on every plan of the batch.
 */
irs_status irs_batch_tune(irs_batch_t batch, const char *cache_path);

/*
 * irs_batch_run -- every map of the batch in one graph launch: for the direct
 * method one persistent kernel drains a device queue of (map, ray tile)
 * items ordered longest map first; for the interpolation the maps' band
 * launches in sequence.  counts[k] is a DEVICE pointer to map k's
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

#ifdef __cplusplus
}
#endif

#endif /* IRS_H */
