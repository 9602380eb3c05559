/*
 * Plain FP64 CPU oracle for the inverse-ray-shooting (IRS) hot path of
 * Zheng et al., "An Improved GPU-Based Ray-Shooting Code for Gravitational
 * Microlensing" (arXiv 2204.10871).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code with the HIP library.
 *
 * Everything is written as the plain definition, in double precision, with no
 * blocking, fusion or reordering beyond what the definitions state:
 *   - O-1, the direct definition: Eq. 6 (deflection with the macro term, the
 *     star sum and the rectangle's negative mass sheet of Appendix A), the lens
 *     mapping beta = theta - alpha (Eq. 4) and the source-pixel binning of the
 *     flow chart (Sec. 2.4, "Calculate the magnification of each pixel").
 *   - O-2, the interpolation step by step (Sec. 2.4): level-1 packing of the
 *     lenses, far-lens Taylor coefficients plus the sheet at the level-2 points,
 *     and level-3 evaluation (near lenses summed exactly + local Taylor series).
 *
 * Geometry (rectangle, ray grid, level-1/2 grids) is derived by the Python side
 * of the oracle from the printed rules and passed in through orc_setup.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double kappa_star;   /* kappa_star : compact (stellar) convergence            */
    double kappa;        /* kappa = kappa_s + kappa_star (Eq. 2)                   */
    double gamma;        /* external shear                                      */
    double a1, a2;       /* lens/image rectangle in theta_1 (Appendix A limits) */
    double b1, b2;       /* lens/image rectangle in theta_2                     */
    int64_t nx, ny;      /* regular ray grid, rays at cell centres              */
    double source_side;  /* S_scale: side of the source map, theta_E units      */
    int64_t npix;        /* pixels per side of the source map                   */
    int64_t sheet;       /* 1: the rectangle's negative mass sheet (Appendix A);
                            2: a circular lens plane's, -kappa_star theta (Eq. 9);
                            0: omit it                                           */
    /* level-1 / level-2 grids (interpolation only) */
    int64_t n1x, n1y;    /* level-1 cells tiling the rectangle                  */
    int64_t q;           /* level-2 points per level-1 cell side                */
} orc_setup;

/* ------------------------------------------------------------------------- */
/* Appendix A: the rectangle's uniform sheet.                                  */
/* ------------------------------------------------------------------------- */

/* p * atan(q / p), whose limit at p = 0 is 0. */
static double p_atan(double p, double q)
{
    if (p == 0.0) return 0.0;
    return p * atan(q / p);
}

/* (p / 2) * ln(num / den), taken as 0 when its prefactor p is 0. */
static double half_p_log(double p, double num, double den)
{
    if (p == 0.0) return 0.0;
    return 0.5 * p * log(num / den);
}

/*
 * The two integrals of Appendix A with A = 1, written out in their printed
 * closed forms: I1 is the theta_1 component (the first closed form of the
 * appendix), I2 the theta_2 component (the second).  With A = kappa/pi they are
 * the deflection of a sheet of POSITIVE density kappa over [a1,a2] x [b1,b2].
 */
void orc_sheet_I(double a1, double a2, double b1, double b2, int64_t n,
                 const double *x, const double *y, double *I1, double *I2)
{
    for (int64_t k = 0; k < n; ++k) {
        const double t1 = x[k], t2 = y[k];
        const double r_a2b2 = (t1 - a2) * (t1 - a2) + (t2 - b2) * (t2 - b2);
        const double r_a1b2 = (t1 - a1) * (t1 - a1) + (t2 - b2) * (t2 - b2);
        const double r_a2b1 = (t1 - a2) * (t1 - a2) + (t2 - b1) * (t2 - b1);
        const double r_a1b1 = (t1 - a1) * (t1 - a1) + (t2 - b1) * (t2 - b1);

        I1[k] = half_p_log(t2 - b2, r_a2b2, r_a1b2)
              - half_p_log(t2 - b1, r_a2b1, r_a1b1)
              + p_atan(t1 - a2, t2 - b2) - p_atan(t1 - a2, t2 - b1)
              + p_atan(t1 - a1, t2 - b1) - p_atan(t1 - a1, t2 - b2);

        I2[k] = half_p_log(t1 - a2, r_a2b2, r_a2b1)
              - half_p_log(t1 - a1, r_a1b2, r_a1b1)
              + p_atan(t2 - b2, t1 - a2) - p_atan(t2 - b2, t1 - a1)
              + p_atan(t2 - b1, t1 - a1) - p_atan(t2 - b1, t1 - a2);
    }
}

/* ------------------------------------------------------------------------- */
/* O-1: the direct definition.                                                 */
/* ------------------------------------------------------------------------- */

/* Ray r of the row-major grid: theta at the centre of grid cell (i, j). */
static void ray_theta(const orc_setup *s, int64_t r, double *t1, double *t2)
{
    const int64_t i = r % s->nx, j = r / s->nx;
    const double dx = (s->a2 - s->a1) / (double)s->nx;
    const double dy = (s->b2 - s->b1) / (double)s->ny;
    *t1 = s->a1 + ((double)i + 0.5) * dx;
    *t2 = s->b1 + ((double)j + 0.5) * dy;
}

/*
 * Eq. 6 at one point: alpha = diag(kappa+gamma, kappa-gamma) theta
 *                           + sum_i m_i (theta - theta_i)/|theta - theta_i|^2
 *                           + alpha_{-kappa_star}(theta),
 * where alpha_{-kappa_star} = -(kappa_star/pi) (I1, I2) is the NEGATIVE sheet that
 * cancels the stars' mean density (the closed forms of Appendix A describe a
 * positive sheet; the sign is flipped here).  On a circular lens plane that
 * contains theta the same sheet deflects by -kappa_star theta (Eq. 9).  A lens
 * exactly at theta contributes nothing and is counted as singular.
 */
static void alpha_direct(const orc_setup *s, int64_t nl, const double *lx,
                         const double *ly, const double *lm, double t1,
                         double t2, double *ax, double *ay, int64_t *nsing)
{
    double sx = 0.0, sy = 0.0;
    for (int64_t i = 0; i < nl; ++i) {
        const double d1 = t1 - lx[i], d2 = t2 - ly[i];
        const double r2 = d1 * d1 + d2 * d2;
        if (r2 == 0.0) { ++*nsing; continue; }
        const double m = lm ? lm[i] : 1.0;
        sx += m * d1 / r2;
        sy += m * d2 / r2;
    }
    double shx = 0.0, shy = 0.0;
    if (s->sheet == 2) {
        shx = -s->kappa_star * t1;
        shy = -s->kappa_star * t2;
    } else if (s->sheet) {
        double I1, I2;
        orc_sheet_I(s->a1, s->a2, s->b1, s->b2, 1, &t1, &t2, &I1, &I2);
        shx = -(s->kappa_star / M_PI) * I1;
        shy = -(s->kappa_star / M_PI) * I2;
    }
    *ax = (s->kappa + s->gamma) * t1 + sx + shx;
    *ay = (s->kappa - s->gamma) * t2 + sy + shy;
}

/* Source pixel of beta: map [-S/2, S/2)^2, floor, row-major iy*npix + ix; -1 off map. */
static int64_t pixel_of(const orc_setup *s, double b1, double b2)
{
    const double dp = s->source_side / (double)s->npix;
    const double fx = floor((b1 + 0.5 * s->source_side) / dp);
    const double fy = floor((b2 + 0.5 * s->source_side) / dp);
    if (!(fx >= 0.0 && fx < (double)s->npix && fy >= 0.0 && fy < (double)s->npix))
        return -1;
    return (int64_t)fy * s->npix + (int64_t)fx;
}

/* Deflection at arbitrary points (Eq. 6). */
void orc_alpha_points(const orc_setup *s, int64_t nl, const double *lx,
                      const double *ly, const double *lm, int64_t n,
                      const double *x, const double *y, double *ax, double *ay,
                      int64_t *nsing_out)
{
    int64_t nsing = 0;
    for (int64_t k = 0; k < n; ++k)
        alpha_direct(s, nl, lx, ly, lm, x[k], y[k], &ax[k], &ay[k], &nsing);
    if (nsing_out) *nsing_out = nsing;
}

/*
 * O-1 over the rays listed in ray_ids (or the contiguous range [first, first+n)
 * when ray_ids is NULL).  Outputs (each nullable): alpha per ray, pixel per ray,
 * counts (accumulated).  stats[0..2] = landed, off-map, singular pairs.
 */
void orc_shoot_direct(const orc_setup *s, int64_t nl, const double *lx,
                      const double *ly, const double *lm, int64_t first,
                      int64_t n, const int64_t *ray_ids, double *ax_out,
                      double *ay_out, int64_t *pix_out, uint32_t *counts,
                      int64_t *stats, int nthreads)
{
    int64_t *pix = pix_out ? pix_out : (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t nsing_total = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nsing_total)
#endif
    for (int64_t k = 0; k < n; ++k) {
        const int64_t r = ray_ids ? ray_ids[k] : first + k;
        double t1, t2, a1, a2;
        int64_t nsing = 0;
        ray_theta(s, r, &t1, &t2);
        alpha_direct(s, nl, lx, ly, lm, t1, t2, &a1, &a2, &nsing);
        nsing_total += nsing;
        if (ax_out) ax_out[k] = a1;
        if (ay_out) ay_out[k] = a2;
        pix[k] = pixel_of(s, t1 - a1, t2 - a2);   /* Eq. 4: beta = theta - alpha */
    }
    int64_t landed = 0, off = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (pix[k] < 0) { ++off; continue; }
        ++landed;
        if (counts) counts[pix[k]] += 1u;
    }
    if (stats) { stats[0] = landed; stats[1] = off; stats[2] = nsing_total; }
    if (!pix_out) free(pix);
}

/* ------------------------------------------------------------------------- */
/* O-2: the three-level-grid interpolation, step by step (Sec. 2.4).           */
/* ------------------------------------------------------------------------- */

/* Level-1 cell of a lens: the rectangle is tiled by n1x x n1y cells. */
static void lens_cell(const orc_setup *s, double x, double y, int64_t *cx, int64_t *cy)
{
    const double w1 = (s->a2 - s->a1) / (double)s->n1x;
    const double h1 = (s->b2 - s->b1) / (double)s->n1y;
    int64_t ix = (int64_t)floor((x - s->a1) / w1);
    int64_t iy = (int64_t)floor((y - s->b1) / h1);
    if (ix < 0) ix = 0;
    if (ix > s->n1x - 1) ix = s->n1x - 1;
    if (iy < 0) iy = 0;
    if (iy > s->n1y - 1) iy = s->n1y - 1;
    *cx = ix;
    *cy = iy;
}

/*
 * "Lenses packed into level-1 grids": a stable counting sort by cell index
 * (row-major cy*n1x + cx).  cell_start has n1x*n1y + 1 entries; perm lists the
 * original lens indices cell by cell, in increasing original order.
 */
void orc_level1(const orc_setup *s, int64_t nl, const double *lx,
                const double *ly, int64_t *cell_start, int64_t *perm)
{
    const int64_t ncell = s->n1x * s->n1y;
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nl > 0 ? nl : 1));
    memset(cell_start, 0, sizeof(int64_t) * (size_t)(ncell + 1));
    for (int64_t i = 0; i < nl; ++i) {
        int64_t cx, cy;
        lens_cell(s, lx[i], ly[i], &cx, &cy);
        cell[i] = cy * s->n1x + cx;
        cell_start[cell[i] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
    memcpy(fill, cell_start, sizeof(int64_t) * (size_t)ncell);
    for (int64_t i = 0; i < nl; ++i) perm[fill[cell[i]]++] = i;
    free(fill);
    free(cell);
}

/* Position of level-2 point (gx, gy): centre of subcell gx, gy of the global
 * level-2 grid, which splits every level-1 cell into q x q subcells. */
static double complex level2_point(const orc_setup *s, int64_t gx, int64_t gy)
{
    const double w2 = (s->a2 - s->a1) / (double)(s->n1x * s->q);
    const double h2 = (s->b2 - s->b1) / (double)(s->n1y * s->q);
    return (s->a1 + ((double)gx + 0.5) * w2) + I * (s->b1 + ((double)gy + 0.5) * h2);
}

/*
 * Complex-analytic form of the sheet (derived from Appendix A; see the tests
 * for the pins).  With F = (I1 - i I2)/pi, inside the rectangle
 * F(z) = conj(z) + G(z), G analytic; the derivatives of G are
 *   G'(z)     = 1 - (i/pi) sum_k s_k Log(z - c_k)
 *   G^(n)(z)  = -(i/pi) sum_k s_k (-1)^n (n-2)! / (z - c_k)^(n-1),  n >= 2,
 * corners c = (a1,b1), (a2,b1), (a2,b2), (a1,b2) with signs s = +1,-1,+1,-1.
 * g[k] = G^(k)(z0)/k! for k = 1..4; g[0] = F(z0).
 */
void orc_sheet_taylor(const orc_setup *s, double complex z0, double complex *g)
{
    const double complex c[4] = { s->a1 + I * s->b1, s->a2 + I * s->b1,
                                  s->a2 + I * s->b2, s->a1 + I * s->b2 };
    const double sg[4] = { 1.0, -1.0, 1.0, -1.0 };
    double t1 = creal(z0), t2 = cimag(z0), I1, I2;
    orc_sheet_I(s->a1, s->a2, s->b1, s->b2, 1, &t1, &t2, &I1, &I2);
    g[0] = (I1 - I * I2) / M_PI;
    /* Log(z - c) with its cut pointing away from the rectangle: up from the
     * top corners (argument in (-3 pi/2, pi/2]), down from the bottom ones
     * (argument in (-pi/2, 3 pi/2]).  Inside the rectangle this is the
     * principal Log; on and just outside the edges (points a rounding step
     * outside) it continues the interior values instead of jumping by 2 pi
     * where the principal cut runs along the top and bottom edges. */
    double complex sum_log = 0.0;
    for (int k = 0; k < 4; ++k) {
        const double u = creal(z0) - creal(c[k]), v = cimag(z0) - cimag(c[k]);
        double th = atan2(v, u);
        if (k >= 2 && th > 0.5 * M_PI) th -= 2.0 * M_PI;
        if (k < 2 && th < -0.5 * M_PI) th += 2.0 * M_PI;
        sum_log += sg[k] * (0.5 * log(u * u + v * v) + I * th);
    }
    g[1] = 1.0 - (I / M_PI) * sum_log;
    static const double fact[5] = { 1.0, 1.0, 2.0, 6.0, 24.0 };
    for (int n = 2; n <= 4; ++n) {
        double complex acc = 0.0;
        for (int k = 0; k < 4; ++k)
            acc += sg[k] * ((n % 2 == 0) ? 1.0 : -1.0) * fact[n - 2] / cpow(z0 - c[k], n - 1);
        g[n] = (-(I / M_PI) * acc) / fact[n];
    }
}

/* The four level-1 cells at the rectangle's corners.  Their level-2 points
 * carry the distant-lens coefficients only; rays there evaluate the sheet in
 * closed form (the sheet's series about a point near a corner does not
 * converge over the subcell: G has log and pole singularities at corners). */
static int is_corner_cell(const orc_setup *s, int64_t cx, int64_t cy)
{
    return (cx == 0 || cx == s->n1x - 1) && (cy == 0 || cy == s->n1y - 1);
}

static int is_near(int64_t cx, int64_t cy, int64_t lcx, int64_t lcy)
{
    return llabs(lcx - cx) <= 1 && llabs(lcy - cy) <= 1;
}

/*
 * "Calculate the deflection angle of level2 grid points": at level-2 point
 * (gx, gy) the distant lenses (outside the 3 x 3 block of level-1 cells around
 * the point's own cell) give
 *   c_j = sum_far m_i (-1)^j / (z0 - z_i)^(j+1),   j = 0..4,
 * and the sheet adds -kappa_star g_j, so that
 *   conj(alpha_far + alpha_sheet)(z0 + h) ~= C0 + sum_{j=1..4} C_j h^j - kappa_star conj(h).
 * Output C[2j] = Re C_j, C[2j + 1] = Im C_j.
 */
static void level2_coef(const orc_setup *s, const double *lx, const double *ly,
                        const double *lm, const int64_t *cell_start, const int64_t *perm,
                        int64_t gx, int64_t gy, double *C)
{
    const double complex z0 = level2_point(s, gx, gy);
    const int64_t cx = gx / s->q, cy = gy / s->q;
    double complex c[5] = { 0, 0, 0, 0, 0 };
    for (int64_t lcy = 0; lcy < s->n1y; ++lcy)
        for (int64_t lcx = 0; lcx < s->n1x; ++lcx) {
            if (is_near(cx, cy, lcx, lcy)) continue;
            const int64_t cell = lcy * s->n1x + lcx;
            for (int64_t p = cell_start[cell]; p < cell_start[cell + 1]; ++p) {
                const int64_t i = perm[p];
                const double m = lm ? lm[i] : 1.0;
                const double complex w = z0 - (lx[i] + I * ly[i]);
                double complex wp = w;     /* w^(j+1) */
                double sign = 1.0;         /* (-1)^j  */
                for (int j = 0; j < 5; ++j) {
                    c[j] += sign * m / wp;
                    wp *= w;
                    sign = -sign;
                }
            }
        }
    double complex g[5] = { 0, 0, 0, 0, 0 };
    if (s->sheet && !is_corner_cell(s, cx, cy)) orc_sheet_taylor(s, z0, g);
    for (int j = 0; j < 5; ++j) {
        const double complex Cj = c[j] - s->kappa_star * g[j];
        C[2 * j] = creal(Cj);
        C[2 * j + 1] = cimag(Cj);
    }
}

/* level2_coef at each requested point (gx[k], gy[k]) into C[k*10 .. k*10 + 9]. */
void orc_level2(const orc_setup *s, int64_t nl, const double *lx,
                const double *ly, const double *lm, const int64_t *cell_start,
                const int64_t *perm, int64_t npts, const int64_t *gx,
                const int64_t *gy, double *C, int nthreads)
{
    (void)nl;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t k = 0; k < npts; ++k)
        level2_coef(s, lx, ly, lm, cell_start, perm, gx[k], gy[k], C + k * 10);
}

/*
 * Level-2 subcell of ray (i, j): the level-2 grid splits [a1,a2] into n1x*q
 * equal columns and the ray sits at the centre of ray cell i, so its column is
 * floor((i + 1/2) n1x q / nx), evaluated exactly in integers.
 */
static void ray_subcell(const orc_setup *s, int64_t r, int64_t *gx, int64_t *gy)
{
    const int64_t i = r % s->nx, j = r / s->nx;
    *gx = ((2 * i + 1) * s->n1x * s->q) / (2 * s->nx);
    *gy = ((2 * j + 1) * s->n1y * s->q) / (2 * s->ny);
}

/*
 * "Calculate the deflection angle of all the light rays (level-3 grids)":
 * near lenses summed exactly, distant lenses and the sheet from the local
 * Taylor series of the ray's level-2 point (coefficients Cp, 10 doubles as
 * produced by orc_level2), plus the macro term.  Rays in the four corner
 * cells take the sheet from its closed form (see is_corner_cell).
 */
static void level3_ray(const orc_setup *s, const double *lx, const double *ly,
                       const double *lm, const int64_t *cell_start, const int64_t *perm,
                       const double *Cp, int64_t r, double *a1_out, double *a2_out,
                       int64_t *pix_out, int64_t *nsing)
{
    double t1, t2;
    int64_t gx, gy;
    ray_theta(s, r, &t1, &t2);
    ray_subcell(s, r, &gx, &gy);
    const int64_t cx = gx / s->q, cy = gy / s->q;

    /* near lenses: exact sum over the 3 x 3 block of level-1 cells */
    double nx_ = 0.0, ny_ = 0.0;
    for (int64_t lcy = cy - 1; lcy <= cy + 1; ++lcy)
        for (int64_t lcx = cx - 1; lcx <= cx + 1; ++lcx) {
            if (lcx < 0 || lcy < 0 || lcx >= s->n1x || lcy >= s->n1y) continue;
            const int64_t cell = lcy * s->n1x + lcx;
            for (int64_t p = cell_start[cell]; p < cell_start[cell + 1]; ++p) {
                const int64_t i = perm[p];
                const double d1 = t1 - lx[i], d2 = t2 - ly[i];
                const double r2 = d1 * d1 + d2 * d2;
                if (r2 == 0.0) { ++*nsing; continue; }
                const double m = lm ? lm[i] : 1.0;
                nx_ += m * d1 / r2;
                ny_ += m * d2 / r2;
            }
        }

    /* distant lenses + sheet: local Taylor series about the level-2 point */
    const double complex z0 = level2_point(s, gx, gy);
    const double complex h = (t1 + I * t2) - z0;
    double complex ca = 0.0, hp = 1.0;
    for (int j = 0; j <= 4; ++j) {
        ca += (Cp[2 * j] + I * Cp[2 * j + 1]) * hp;
        hp *= h;
    }
    if (s->sheet) {
        if (is_corner_cell(s, cx, cy)) {
            double I1, I2;
            orc_sheet_I(s->a1, s->a2, s->b1, s->b2, 1, &t1, &t2, &I1, &I2);
            ca += -(s->kappa_star / M_PI) * (I1 - I * I2);
        } else {
            ca += -s->kappa_star * conj(h);
        }
    }
    /* conj(ca) is the far + sheet deflection */
    const double a1 = (s->kappa + s->gamma) * t1 + nx_ + creal(ca);
    const double a2 = (s->kappa - s->gamma) * t2 + ny_ - cimag(ca);
    *a1_out = a1;
    *a2_out = a2;
    *pix_out = pixel_of(s, t1 - a1, t2 - a2);
}

/* Counts and landed / off-map totals of the per-ray pixels pix[0..n). */
static void bin_pixels(int64_t n, const int64_t *pix, uint32_t *counts, int64_t nsing,
                       int64_t *stats)
{
    int64_t landed = 0, off = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (pix[k] < 0) { ++off; continue; }
        ++landed;
        if (counts) counts[pix[k]] += 1u;
    }
    if (stats) { stats[0] = landed; stats[1] = off; stats[2] = nsing; }
}

/*
 * Level-3 evaluation of the rays listed in ray_ids (or [first, first+n)) with
 * the coefficients of the whole level-2 grid, Ccoef: point (gx, gy) at index
 * gy*(n1x*q) + gx, 10 doubles each as produced by orc_level2.
 */
void orc_shoot_interp(const orc_setup *s, int64_t nl, const double *lx,
                      const double *ly, const double *lm,
                      const int64_t *cell_start, const int64_t *perm,
                      const double *Ccoef, int64_t first, int64_t n,
                      const int64_t *ray_ids, double *ax_out, double *ay_out,
                      int64_t *pix_out, uint32_t *counts, int64_t *stats,
                      int nthreads)
{
    (void)nl;
    int64_t *pix = pix_out ? pix_out : (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    const int64_t ngx = s->n1x * s->q;
    int64_t nsing_total = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nsing_total)
#endif
    for (int64_t k = 0; k < n; ++k) {
        const int64_t r = ray_ids ? ray_ids[k] : first + k;
        int64_t gx, gy, nsing = 0;
        double a1, a2;
        ray_subcell(s, r, &gx, &gy);
        level3_ray(s, lx, ly, lm, cell_start, perm, Ccoef + (gy * ngx + gx) * 10, r, &a1, &a2,
                   &pix[k], &nsing);
        nsing_total += nsing;
        if (ax_out) ax_out[k] = a1;
        if (ay_out) ay_out[k] = a2;
    }
    bin_pixels(n, pix, counts, nsing_total, stats);
    if (!pix_out) free(pix);
}

/*
 * The same level-3 evaluation for rays listed in ray_ids (or [first, first+n)),
 * each taking the coefficients of its own level-2 point from the distant-lens
 * sum of orc_level2 computed on the spot.  Results equal orc_shoot_interp's
 * with the whole level-2 grid; the cost is one distant-lens sum per ray, so
 * rays of maps whose level-2 grid is too large to build can be checked.
 */
void orc_shoot_interp_rays(const orc_setup *s, int64_t nl, const double *lx,
                           const double *ly, const double *lm,
                           const int64_t *cell_start, const int64_t *perm, int64_t first,
                           int64_t n, const int64_t *ray_ids, double *ax_out,
                           double *ay_out, int64_t *pix_out, uint32_t *counts,
                           int64_t *stats, int nthreads)
{
    (void)nl;
    int64_t *pix = pix_out ? pix_out : (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t nsing_total = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nsing_total)
#endif
    for (int64_t k = 0; k < n; ++k) {
        const int64_t r = ray_ids ? ray_ids[k] : first + k;
        int64_t gx, gy, nsing = 0;
        double C[10], a1, a2;
        ray_subcell(s, r, &gx, &gy);
        level2_coef(s, lx, ly, lm, cell_start, perm, gx, gy, C);
        level3_ray(s, lx, ly, lm, cell_start, perm, C, r, &a1, &a2, &pix[k], &nsing);
        nsing_total += nsing;
        if (ax_out) ax_out[k] = a1;
        if (ay_out) ay_out[k] = a2;
    }
    bin_pixels(n, pix, counts, nsing_total, stats);
    if (!pix_out) free(pix);
}

/* orc_sheet_taylor at z0 = x + i y, outputs interleaved (Re, Im) of g_0..g_4. */
void orc_sheet_taylor_xy(const orc_setup *s, double x, double y, double *out)
{
    double complex g[5];
    orc_sheet_taylor(s, x + I * y, g);
    for (int k = 0; k < 5; ++k) {
        out[2 * k] = creal(g[k]);
        out[2 * k + 1] = cimag(g[k]);
    }
}

/* ------------------------------------------------------------------------- */
/* Far field at arbitrary points (the learned interpolant's exact samples).    */
/* ------------------------------------------------------------------------- */

/*
 * Analytic far field of cell (cx, cy) at points z = x + i y, by the plain
 * definition: the distant lenses (outside the 3 x 3 block around the cell)
 * give A(z) = sum m_i / (z - z_i) and A'(z) = -sum m_i / (z - z_i)^2; outside
 * the four corner cells the analytic part of the sheet is added,
 * -kappa_star G(z) and -kappa_star G'(z), with G(z) = F(z) - conj(z) (the sheet's
 * remaining term -kappa_star conj(z) is the ray's own, exactly linear).  So
 * conj(alpha_far + alpha_sheet)(z) = A(z) - kappa_star conj(z) in non-corner
 * cells and A(z) - kappa_star F(z) in corner cells.
 * out[4k..4k+3] = Re A, Im A, Re A', Im A'.
 */
void orc_far_point(const orc_setup *s, int64_t nl, const double *lx, const double *ly,
                   const double *lm, const int64_t *cell_start, const int64_t *perm,
                   int64_t npts, const int64_t *pcx, const int64_t *pcy, const double *px,
                   const double *py, double *out, int nthreads)
{
    (void)nl;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t k = 0; k < npts; ++k) {
        const double complex z = px[k] + I * py[k];
        const int64_t cx = pcx[k], cy = pcy[k];
        double complex A = 0.0, dA = 0.0;
        for (int64_t lcy = 0; lcy < s->n1y; ++lcy)
            for (int64_t lcx = 0; lcx < s->n1x; ++lcx) {
                if (is_near(cx, cy, lcx, lcy)) continue;
                const int64_t cell = lcy * s->n1x + lcx;
                for (int64_t p = cell_start[cell]; p < cell_start[cell + 1]; ++p) {
                    const int64_t i = perm[p];
                    const double m = lm ? lm[i] : 1.0;
                    const double complex w = z - (lx[i] + I * ly[i]);
                    A += m / w;
                    dA -= m / (w * w);
                }
            }
        if (s->sheet && !is_corner_cell(s, cx, cy)) {
            double complex g[5];
            orc_sheet_taylor(s, z, g);
            A -= s->kappa_star * (g[0] - conj(z));
            dA -= s->kappa_star * g[1];
        }
        out[4 * k] = creal(A);
        out[4 * k + 1] = cimag(A);
        out[4 * k + 2] = creal(dA);
        out[4 * k + 3] = cimag(dA);
    }
}
