// Learned interpolant of the distant-lens field: the library's extension of
// the interpolation of Sec. 2.4 (the formulas are stated with irs_learn in
// irs.h).  The nearby lenses stay exact; the distant lenses and the analytic
// part of the sheet, an analytic function A(z) inside each level-1 cell, are
// known exactly at the corners of a coarse grid of squares and interpolated in
// between by I(z) + sigma * sum_k L_k(h) D_k, L from a small network.  The
// rays take L from the network's outputs tabulated at 33 x 33 nodes of the
// unit square, blended bilinearly.
//
// Kernels
//   k_learn_corners   A, A' at every corner of the squares of a band of cells
//   k_learn_samples   exact samples (h, D, T = (A - I)/sigma, sigma)
//   k_mlp_pack        FP32 parameters -> BF16 MFMA operand fragments
//   k_mlp_fwd         network outputs at given offsets (inference kernel; also
//                     the rays' table of weights)
//   k_mlp_train       forward, loss gradient and backward of a batch
//   k_mlp_wgrad       weight and bias gradients, per chunk of the batch
//   k_mlp_reduce      chunk sums in fixed order, batch loss
//   k_adam            Adam step on the FP32 parameters
//   k_learn_err       per-sample validation errors
//   k_ltab_eval       the tabulated weights at given offsets
//   k_learn_cols      per ray column: square column and level-1 column
//   k_level3_learned  rays: near lenses exact, learned distant field, macro
//                     term, beta, pixel, binning by runs (the rectangle's
//                     corner cells in k_level3_learned_corner)
//
// Matrix-core layout (v_mfma_f32_32x32x16_bf16, one wave): A is 32 x 16, lane
// l holds A[l%32][8(l/32) + v]; B is 16 x 32, lane l holds B[8(l/32) + v][l%32];
// the 32 x 32 result D in 16 registers, D[8(r/4) + 4(l/32) + r%4][l%32].  The
// network runs transposed: rows are units (M), columns are samples (N), so a
// layer's result registers are already the next layer's B operand once the
// K index of the weights is permuted the same way; no LDS round trip between
// layers.  A wave carries 64 samples as two 32-sample column blocks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "level2.hpp"

namespace irs {

namespace {

constexpr int kW = 64;                // wavefront
constexpr int kNF = IRS_LEARN_NFREQ;  // 64 frequencies -> 128 features
constexpr int kHd = 128;              // hidden width
constexpr int kNO = 16;               // outputs (8 complex weights)
constexpr int kNP = IRS_LEARN_NPARAMS;
constexpr int kNFld = IRS_LEARN_FIELDS;

__host__ __device__ constexpr int offW(int l) { return l * (kHd * kHd + kHd); }   // W_{l+1}
__host__ __device__ constexpr int offB(int l) { return offW(l) + kHd * kHd; }      // b_{l+1}
constexpr int kOffW5 = 4 * (kHd * kHd + kHd);
constexpr int kOffB5 = kOffW5 + kNO * kHd;
static_assert(kOffB5 + kNO == kNP, "parameter layout");

// operand fragments: 16 bytes (8 BF16) per lane
constexpr int kFragHidden = 4 * 8 * kW;                  // 4 row blocks x 8 K-steps
constexpr int kFragHead = 8 * kW;                        // 1 row block (16 + 16 zero rows)
constexpr int kFragFwd = 4 * kFragHidden + kFragHead;    // 139264 bytes
constexpr int kFragBwd = 3 * kFragHidden + 4 * kW;       // W2..W4 and W5 transposed
constexpr int kBias = 4 * kHd + kNO;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16 rounded to nearest even (the hardware conversion)
__device__ inline uint16_t f2bf(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
// two values in one word, a in the low half (one packed conversion)
__device__ inline uint32_t pack2(float a, float b)
{
    const bf16x2 v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
}

__device__ inline f32x16 mfma(const uint4 &a, const uint4 &b, const f32x16 &c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// column (input unit) held in slot v by lane half h at K-step t: the input
// layer takes the features in natural order; later layers take the previous
// result registers, whose units follow the result layout
__host__ __device__ inline int kcol(bool first, int t, int h, int v)
{
    return first ? 16 * t + 8 * h + v : 16 * t + 8 * (v / 4) + 4 * h + v % 4;
}
// unit held by result register r of row block mb in lane half h
__host__ __device__ inline int drow(int mb, int r, int h) { return 32 * mb + 8 * (r / 4) + 4 * h + r % 4; }

// ---------------------------------------------------------------------------
// The network on one 32-sample column block nb of a wave.  Sample 32 nb + n
// is owned by lane 32 nb + n; lanes n and n + 32 both carry it through the
// matrix products (each holds half of every operand column).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void features(const float *__restrict__ freq, float hx, float hy, uint4 B[8])
{
    const int h = (threadIdx.x % kW) / 32;
    const float px = hx - 0.5f, py = hy - 0.5f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        float s[8], c[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int j = 16 * t + 8 * h + v;
            const float a = fmaf(freq[2 * j], px, freq[2 * j + 1] * py);
            const float r = a - rintf(a);                 // revolutions, |r| <= 1/2
            s[v] = __builtin_amdgcn_sinf(r);              // sin(2 pi r)
            c[v] = __builtin_amdgcn_cosf(r);
        }
        B[t] = make_uint4(pack2(s[0], s[1]), pack2(s[2], s[3]), pack2(s[4], s[5]), pack2(s[6], s[7]));
        B[t + 4] = make_uint4(pack2(c[0], c[1]), pack2(c[2], c[3]), pack2(c[4], c[5]), pack2(c[6], c[7]));
    }
}

// one hidden layer: B (8 K-steps) -> relu(W B + b) -> B; mask: bit 16 mb + r
// set where result register r of row block mb is positive
template <bool SAVE>
__device__ __forceinline__ void hidden_layer(const uint4 *__restrict__ wf, const float *__restrict__ bias,
                                             uint4 B[8], uint64_t &mask)
{
    const int lane = threadIdx.x % kW, h = lane / 32;
    f32x16 acc[4];
    // the products accumulate onto the bias (its loads then overlap them)
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[ob][r] = bias[drow(ob, r, h)];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) acc[ob] = mfma(wf[(ob * 8 + t) * kW + lane], B[t], acc[ob]);
        asm volatile("" ::: "memory");      // keep the fragment loads of later steps here
    }
    if (SAVE) mask = 0;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            float o[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                o[v] = fmaxf(acc[mb][8 * j + v], 0.0f);
                if (SAVE && o[v] > 0.0f) mask |= 1ull << (16 * mb + 8 * j + v);
            }
            B[2 * mb + j] = make_uint4(pack2(o[0], o[1]), pack2(o[2], o[3]), pack2(o[4], o[5]),
                                       pack2(o[6], o[7]));
        }
}

// head: the owner lanes (h == nb) receive their sample's 16 outputs in y
__device__ __forceinline__ void head_layer(const uint4 *__restrict__ wf, const float *__restrict__ b5,
                                           const uint4 B[8], int nb, float y[kNO])
{
    const int lane = threadIdx.x % kW, h = lane / 32;
    f32x16 o;
#pragma unroll
    for (int r = 0; r < 16; ++r) o[r] = 0.0f;
#pragma unroll
    for (int t = 0; t < 8; ++t) o = mfma(wf[t * kW + lane], B[t], o);
    // registers 0..7 hold rows 8(r/4) + 4h + r%4; lane l ^ 32 holds the others
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const float rcv = __shfl_xor(o[r], 32);
        const int r0 = 8 * (r / 4) + r % 4;        // row of half 0
        if (h == nb) {
            y[r0] = (h ? rcv : o[r]) + b5[r0];
            y[r0 + 4] = (h ? o[r] : rcv) + b5[r0 + 4];
        }
    }
}

// inference: 64 offsets, one per lane, in; the lane's 16 outputs out
__device__ __forceinline__ void mlp_forward(const uint4 *__restrict__ wf, const float *__restrict__ bias,
                                            const float *__restrict__ freq, float hx, float hy,
                                            float y[kNO])
{
    const int n = threadIdx.x % 32;
#pragma unroll 1
    for (int nb = 0; nb < 2; ++nb) {
        uint4 B[8];
        features(freq, __shfl(hx, 32 * nb + n), __shfl(hy, 32 * nb + n), B);
        uint64_t m;
#pragma unroll 1
        for (int L = 0; L < 4; ++L) hidden_layer<false>(wf + L * kFragHidden, bias + L * kHd, B, m);
        head_layer(wf + 4 * kFragHidden, bias + 4 * kHd, B, nb, y);
    }
}

// ---------------------------------------------------------------------------
// Squares: base interpolant and local data (same code for samples and rays)
// ---------------------------------------------------------------------------
struct LearnGeom {
    int32_t qc;            // squares per cell side
    int32_t pad_;
    double sx, sy;         // square sides: I_x/(n1x qc), I_y/(n1y qc)
};

__device__ __forceinline__ double corner_x(const DevGeom &g, const LearnGeom &lg, int64_t gxc)
{
#pragma clang fp contract(off)
    return g.a1 + (double)gxc * lg.sx;
}
__device__ __forceinline__ double corner_y(const DevGeom &g, const LearnGeom &lg, int64_t gyc)
{
#pragma clang fp contract(off)
    return g.b1 + (double)gyc * lg.sy;
}

struct Sq {
    double Ir, Ii;         // base interpolant
    double sigma;
    float D[16];           // Re, Im of D_0..D_7
};

// C: the four corners' (Re A, Im A, Re A', Im A'), order lower-left,
// lower-right, upper-left, upper-right; X0/X1, Y0/Y1 their coordinates.
// The base interpolant at (x, y), in-square offset (hx, hy).
__device__ __forceinline__ void square_base(const double C[4][4], double X0, double X1, double Y0,
                                            double Y1, double x, double y, double hx, double hy,
                                            double &Ir, double &Ii)
{
    const double zx[4] = {X0, X1, X0, X1}, zy[4] = {Y0, Y0, Y1, Y1};
    const double w[4] = {(1 - hx) * (1 - hy), hx * (1 - hy), (1 - hx) * hy, hx * hy};
    Ir = 0.0;
    Ii = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double ux = x - zx[c], uy = y - zy[c];
        Ir += w[c] * (C[c][0] + (C[c][2] * ux - C[c][3] * uy));
        Ii += w[c] * (C[c][1] + (C[c][2] * uy + C[c][3] * ux));
    }
}

// The square's local data D (normalised) and its size sigma.
__device__ __forceinline__ void square_local(const double C[4][4], double X0, double X1, double Y0,
                                             double Y1, const LearnGeom &lg, float D[16],
                                             double &sigma)
{
    const double zx[4] = {X0, X1, X0, X1}, zy[4] = {Y0, Y0, Y1, Y1};
    double mAr = 0, mAi = 0, mdr = 0, mdi = 0, mzx = 0, mzy = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        mAr += C[c][0]; mAi += C[c][1]; mdr += C[c][2]; mdi += C[c][3];
        mzx += zx[c]; mzy += zy[c];
    }
    mAr *= 0.25; mAi *= 0.25; mdr *= 0.25; mdi *= 0.25; mzx *= 0.25; mzy *= 0.25;
    const double s = 0.5 * (lg.sx + lg.sy);
    // the data of corner c (delta_c, eps_c), formed twice (for sigma, then
    // scaled) so that the 16 values are never held at once; sigma is the
    // root of the largest squared size (the root is monotonic: the same
    // value as the largest root)
    auto data = [&](int c, double dd[4]) {
        dd[0] = (C[c][2] - mdr) * s;
        dd[1] = (C[c][3] - mdi) * s;
        const double vx = zx[c] - mzx, vy = zy[c] - mzy;
        dd[2] = C[c][0] - mAr - (mdr * vx - mdi * vy);
        dd[3] = C[c][1] - mAi - (mdr * vy + mdi * vx);
    };
    double sig2 = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double dd[4];
        data(c, dd);
        sig2 = fmax(sig2, dd[0] * dd[0] + dd[1] * dd[1]);
        sig2 = fmax(sig2, dd[2] * dd[2] + dd[3] * dd[3]);
    }
    sigma = fmax(sqrt(sig2), 1e-280);
    const double is = 1.0 / sigma;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double dd[4];
        data(c, dd);
        D[2 * c] = (float)(dd[0] * is);
        D[2 * c + 1] = (float)(dd[1] * is);
        D[8 + 2 * c] = (float)(dd[2] * is);
        D[8 + 2 * c + 1] = (float)(dd[3] * is);
    }
}

__device__ __forceinline__ void square_eval(const double C[4][4], double X0, double X1, double Y0,
                                            double Y1, const LearnGeom &lg, double x, double y,
                                            double hx, double hy, Sq &o)
{
    square_base(C, X0, X1, Y0, Y1, x, y, hx, hy, o.Ir, o.Ii);
    square_local(C, X0, X1, Y0, Y1, lg, o.D, o.sigma);
}

// sum_k L_k D_k with L_k = y_2k + i y_2k+1
__device__ __forceinline__ void combine(const float y[kNO], const float D[16], float &pr, float &pi)
{
    pr = 0.0f;
    pi = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        pr = fmaf(y[2 * k], D[2 * k], fmaf(-y[2 * k + 1], D[2 * k + 1], pr));
        pi = fmaf(y[2 * k], D[2 * k + 1], fmaf(y[2 * k + 1], D[2 * k], pi));
    }
}

// ---------------------------------------------------------------------------
// The weights L(h) as the rays take them: the network's 16 outputs at the
// (kLTab + 1)^2 nodes (a/kLTab, b/kLTab) of the unit square (node b (kLTab+1)
// + a), blended bilinearly between the four nodes around h.  L depends on h
// alone, so the network runs once per node instead of once per ray; the
// blend's own error is far inside the network's (its features turn slowly
// over the square, and the validation measures the blended weights).
// ---------------------------------------------------------------------------
constexpr int kLTab = 32;
constexpr int kLNodes = (kLTab + 1) * (kLTab + 1);

// value (o, node k) = t[k NS + o OS]; h outside [0, 1] (rounding) is clamped
template <int NS, int OS>
__device__ __forceinline__ void ltab_blend(const float *__restrict__ t, float hx, float hy,
                                           float y[kNO])
{
    const float u = fminf(fmaxf(hx, 0.0f), 1.0f) * (float)kLTab;
    const float v = fminf(fmaxf(hy, 0.0f), 1.0f) * (float)kLTab;
    const int a = min((int)u, kLTab - 1), b = min((int)v, kLTab - 1);
    const float fu = u - (float)a, fv = v - (float)b;
    const float w00 = (1.0f - fu) * (1.0f - fv), w10 = fu * (1.0f - fv);
    const float w01 = (1.0f - fu) * fv, w11 = fu * fv;
    const float *t00 = t + (b * (kLTab + 1) + a) * NS;
    const float *t01 = t00 + (kLTab + 1) * NS;
#pragma unroll
    for (int o = 0; o < kNO; ++o)
        y[o] = w00 * t00[o * OS] + w10 * t00[NS + o * OS] + w01 * t01[o * OS] +
               w11 * t01[NS + o * OS];
}

// sum_k L_k D_k with L the table's blend at (hx, hy) (combine's arithmetic on
// ltab_blend's weights, one weight pair at a time)
template <int NS, int OS>
__device__ __forceinline__ void ltab_combine(const float *__restrict__ t, float hx, float hy,
                                             const float D[16], float &pr, float &pi)
{
    const float u = fminf(fmaxf(hx, 0.0f), 1.0f) * (float)kLTab;
    const float v = fminf(fmaxf(hy, 0.0f), 1.0f) * (float)kLTab;
    const int a = min((int)u, kLTab - 1), b = min((int)v, kLTab - 1);
    const float fu = u - (float)a, fv = v - (float)b;
    const float w00 = (1.0f - fu) * (1.0f - fv), w10 = fu * (1.0f - fv);
    const float w01 = (1.0f - fu) * fv, w11 = fu * fv;
    const float *t00 = t + (b * (kLTab + 1) + a) * NS;
    const float *t01 = t00 + (kLTab + 1) * NS;
    auto at = [&](int o) {
        return w00 * t00[o * OS] + w10 * t00[NS + o * OS] + w01 * t01[o * OS] +
               w11 * t01[NS + o * OS];
    };
    pr = 0.0f;
    pi = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float yr = at(2 * k), yi = at(2 * k + 1);
        pr = fmaf(yr, D[2 * k], fmaf(-yi, D[2 * k + 1], pr));
        pi = fmaf(yr, D[2 * k + 1], fmaf(yi, D[2 * k], pi));
    }
}

// ---------------------------------------------------------------------------
// Exact distant field of a cell at a point: the cell's expansion (lenses
// outside the (2R+1)^2 block), the ring lenses, and -kappa_* G (outside the
// corner cells).  L: summed expansion coefficients of the cell.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool corner_cell_l(const DevGeom &g, int64_t cx, int64_t cy)
{
    return (cx == 0 || cx == g.n1x - 1) && (cy == 0 || cy == g.n1y - 1);
}

template <bool UNIT, int P>
__device__ void far_at(const DevGeom &g, const double (*L)[2], int32_t cx, int32_t cy, double x,
                       double y, const double *__restrict__ lx, const double *__restrict__ ly,
                       const double *__restrict__ lm, const int32_t *__restrict__ cell_start,
                       double out[4])
{
    const double sc = fmax(g.w1, g.h1), isc = 1.0 / sc;
    const double zcr = g.a1 + ((double)cx + 0.5) * g.w1;
    const double zci = g.b1 + ((double)cy + 0.5) * g.h1;
    const double dr = (x - zcr) * isc, di = (y - zci) * isc;
    // Horner: A = sum L_n d^n, A' = sum n L_n d^(n-1)
    double Ar = L[P - 1][0], Ai = L[P - 1][1];
    double Dr = (double)(P - 1) * Ar, Di = (double)(P - 1) * Ai;
#pragma unroll 4
    for (int n = P - 2; n >= 0; --n) {
        const double tr = Ar * dr - Ai * di;
        Ai = Ar * di + Ai * dr + L[n][1];
        Ar = tr + L[n][0];
        if (n >= 1) {
            const double ur = Dr * dr - Di * di;
            Di = Dr * di + Di * dr + (double)n * L[n][1];
            Dr = ur + (double)n * L[n][0];
        }
    }
    Ar *= isc; Ai *= isc;
    Dr *= isc * isc; Di *= isc * isc;
    // ring lenses: inside the (2R+1)^2 block, outside the 3 x 3 block
    const int32_t yl = max(0, cy - kRing), yh = min(g.n1y - 1, cy + kRing);
    for (int32_t row = yl; row <= yh; ++row) {
        const bool mid = abs(row - cy) <= 1;
        for (int seg = 0; seg < (mid ? 2 : 1); ++seg) {
            int32_t xa, xb;
            if (!mid) { xa = cx - kRing; xb = cx + kRing; }
            else if (seg == 0) { xa = cx - kRing; xb = cx - 2; }
            else { xa = cx + 2; xb = cx + kRing; }
            xa = max(xa, 0);
            xb = min(xb, g.n1x - 1);
            if (xa > xb) continue;
            const int32_t pb = cell_start[row * g.n1x + xa];
            const int32_t pe = cell_start[row * g.n1x + xb + 1];
            for (int32_t pl = pb; pl < pe; ++pl) {
                const double wr = x - lx[pl], wi = y - ly[pl];
                const double inv = 1.0 / (wr * wr + wi * wi);
                const double m = UNIT ? 1.0 : lm[pl];
                const double ur = wr * inv, ui = -wi * inv;          // 1/(z - z_i)
                Ar += m * ur;
                Ai += m * ui;
                Dr -= m * (ur * ur - ui * ui);
                Di -= m * (2.0 * ur * ui);
            }
        }
    }
    if (g.sheet && !corner_cell_l(g, cx, cy)) {
        // G = F - conj(z), F = (I1 - i I2)/pi;  G' = 1 - (i/pi) sum_k s_k Log(z - c_k)
        double I1, I2;
        sheet_unit(g, x, y, I1, I2);
        const double ipi = 1.0 / M_PI;
        const double Gr = I1 * ipi - x, Gi = -I2 * ipi + y;
        double lr = 0.0, li = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double a = (c == 0 || c == 3) ? g.a1 : g.a2;
            const double b = (c < 2) ? g.b1 : g.b2;
            const double sgn = (c == 0 || c == 2) ? 1.0 : -1.0;
            const double u = x - a, v = y - b;
            lr += sgn * 0.5 * log(u * u + v * v);
            li += sgn * log_arg(u, v, c >= 2);
        }
        const double G1r = 1.0 + li * ipi, G1i = -lr * ipi;
        Ar -= g.kappa_star * Gr;
        Ai -= g.kappa_star * Gi;
        Dr -= g.kappa_star * G1r;
        Di -= g.kappa_star * G1i;
    }
    out[0] = Ar;
    out[1] = Ai;
    out[2] = Dr;
    out[3] = Di;
}

constexpr int kThreads = 256;
constexpr int kCells = kThreads / kW;       // cells per workgroup (as the expansion kernel)

// sum the chunks' partial expansions of the block's cells, in chunk order
template <int P>
__device__ void sum_partials(const DevGeom &g, const double *__restrict__ part, int32_t cy, int32_t cy0,
                             int32_t cx0, int32_t nchunk, double (*sL)[P][2])
{
    for (int e = threadIdx.x; e < kCells * P * 2; e += kThreads) {
        const int w = e / (P * 2), n = (e / 2) % P, comp = e % 2;
        const int32_t cx = cx0 + w;
        double acc = 0.0;
        if (cx < g.n1x) {
            const double *src = part + (((int64_t)(cy - cy0) * g.n1x + cx) * nchunk * P + n) * 2 + comp;
            for (int k = 0; k < nchunk; ++k) acc += src[(int64_t)k * P * 2];
        }
        sL[w][n][comp] = acc;
    }
}

template <bool UNIT, int P>
__global__ __launch_bounds__(kThreads) void k_learn_corners(
    DevGeom g, LearnGeom lg, const double *__restrict__ lx, const double *__restrict__ ly,
    const double *__restrict__ lm, const int32_t *__restrict__ cell_start, int32_t cy0, int32_t nxb,
    int32_t nchunk, const double *__restrict__ part, double *__restrict__ corner)
{
    __shared__ double sL[kCells][P][2];
    const int32_t cy = cy0 + (int32_t)(blockIdx.x / (uint32_t)nxb);
    const int32_t cx0 = (int32_t)(blockIdx.x % (uint32_t)nxb) * kCells;
    sum_partials<P>(g, part, cy, cy0, cx0, nchunk, sL);
    __syncthreads();
    const int q1 = lg.qc + 1, npts = q1 * q1;
    for (int pp = threadIdx.x; pp < kCells * npts; pp += kThreads) {
        const int w = pp / npts, pt = pp % npts;
        const int32_t cx = cx0 + w;
        if (cx >= g.n1x) continue;
        const int a = pt % q1, b = pt / q1;
        const double x = corner_x(g, lg, (int64_t)cx * lg.qc + a);
        const double y = corner_y(g, lg, (int64_t)cy * lg.qc + b);
        double o[4];
        far_at<UNIT, P>(g, sL[w], cx, cy, x, y, lx, ly, lm, cell_start, o);
        double *dst = corner + (((int64_t)(cy - cy0) * g.n1x + cx) * npts + pt) * 4;
        dst[0] = o[0];
        dst[1] = o[1];
        dst[2] = o[2];
        dst[3] = o[3];
    }
}

// counter-based uniform in [0, 1): splitmix64 of (seed, index, stream)
__device__ __forceinline__ double u01(uint64_t seed, uint64_t idx, uint32_t k)
{
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + idx * 4ull + k + 1ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ void load_corners(const double *__restrict__ corner, int64_t cell, int q1,
                                             int a, int b, double C[4][4])
{
    const double *base = corner + cell * (int64_t)q1 * q1 * 4;
    const int idx[4] = {b * q1 + a, b * q1 + a + 1, (b + 1) * q1 + a, (b + 1) * q1 + a + 1};
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k) C[c][k] = base[idx[c] * 4 + k];
}

template <bool UNIT, int P>
__global__ __launch_bounds__(kThreads) void k_learn_samples(
    DevGeom g, LearnGeom lg, const double *__restrict__ lx, const double *__restrict__ ly,
    const double *__restrict__ lm, const int32_t *__restrict__ cell_start, int32_t cy0, int32_t nxb,
    int32_t nchunk, const double *__restrict__ part, const double *__restrict__ corner,
    int32_t per_cell, uint64_t seed, int64_t n_out, float *__restrict__ out)
{
    __shared__ double sL[kCells][P][2];
    const int32_t cy = cy0 + (int32_t)(blockIdx.x / (uint32_t)nxb);
    const int32_t cx0 = (int32_t)(blockIdx.x % (uint32_t)nxb) * kCells;
    sum_partials<P>(g, part, cy, cy0, cx0, nchunk, sL);
    __syncthreads();
    const int q1 = lg.qc + 1;
    for (int k = threadIdx.x; k < kCells * per_cell; k += kThreads) {
        const int w = k / per_cell;
        const int32_t cx = cx0 + w;
        if (cx >= g.n1x) continue;
        const int64_t cell = (int64_t)(cy - cy0) * g.n1x + cx;
        const int64_t sid = cell * per_cell + k % per_cell;
        const uint64_t gid = ((uint64_t)cy * (uint64_t)g.n1x + (uint64_t)cx) * (uint64_t)per_cell +
                             (uint64_t)(k % per_cell);
        const int a = min(lg.qc - 1, (int)(u01(seed, gid, 0) * lg.qc));
        const int b = min(lg.qc - 1, (int)(u01(seed, gid, 1) * lg.qc));
        const double hx = u01(seed, gid, 2), hy = u01(seed, gid, 3);
        const int64_t gxc = (int64_t)cx * lg.qc + a, gyc = (int64_t)cy * lg.qc + b;
        const double X0 = corner_x(g, lg, gxc), X1 = corner_x(g, lg, gxc + 1);
        const double Y0 = corner_y(g, lg, gyc), Y1 = corner_y(g, lg, gyc + 1);
        const double x = X0 + hx * lg.sx, y = Y0 + hy * lg.sy;
        double A[4];
        far_at<UNIT, P>(g, sL[w], cx, cy, x, y, lx, ly, lm, cell_start, A);
        double C[4][4];
        load_corners(corner, cell, q1, a, b, C);
        Sq sq;
        square_eval(C, X0, X1, Y0, Y1, lg, x, y, hx, hy, sq);
        const double is = 1.0 / sq.sigma;
        float f[kNFld];
        f[0] = (float)hx;
        f[1] = (float)hy;
#pragma unroll
        for (int e = 0; e < 16; ++e) f[2 + e] = sq.D[e];
        f[18] = (float)((A[0] - sq.Ir) * is);
        f[19] = (float)((A[1] - sq.Ii) * is);
        f[20] = (float)sq.sigma;
        f[21] = (float)cx;
        f[22] = (float)cy;
        f[23] = (float)(b * lg.qc + a);
#pragma unroll
        for (int e = 0; e < kNFld; ++e) out[(int64_t)e * n_out + sid] = f[e];
    }
}

// ---------------------------------------------------------------------------
// Parameters -> fragments
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_mlp_pack(const float *__restrict__ theta,
                                                       uint16_t *__restrict__ wf,
                                                       uint16_t *__restrict__ wb)
{
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t nf = (int64_t)kFragFwd * 8, nb = (int64_t)kFragBwd * 8;
    if (e < nf) {
        const int frag = (int)(e / 8), v = (int)(e % 8);
        const int lane = frag % kW, h = lane / 32, m = lane % 32;
        float val = 0.0f;
        if (frag < 4 * kFragHidden) {
            const int L = frag / kFragHidden, rem = frag % kFragHidden / kW;
            const int ob = rem / 8, t = rem % 8;
            val = theta[offW(L) + (32 * ob + m) * kHd + kcol(L == 0, t, h, v)];
        } else {
            const int t = (frag - 4 * kFragHidden) / kW;
            if (m < kNO) val = theta[kOffW5 + m * kHd + kcol(false, t, h, v)];
        }
        wf[e] = f2bf(val);
    } else if (wb && e < nf + nb) {
        const int64_t eb = e - nf;
        const int frag = (int)(eb / 8), v = (int)(eb % 8);
        const int lane = frag % kW, h = lane / 32, m = lane % 32;
        float val;
        if (frag < 3 * kFragHidden) {
            // W_{L+2} transposed: rows = input units 32 ib + m, K = output units
            const int L = frag / kFragHidden, rem = frag % kFragHidden / kW;
            const int ib = rem / 8, t = rem % 8;
            val = theta[offW(L + 1) + kcol(false, t, h, v) * kHd + 32 * ib + m];
        } else {
            const int ib = (frag - 3 * kFragHidden) / kW;
            val = theta[kOffW5 + kcol(false, 0, h, v) * kHd + 32 * ib + m];
        }
        wb[eb] = f2bf(val);
    }
}

// ---------------------------------------------------------------------------
// Inference over given offsets
// ---------------------------------------------------------------------------
struct MlpSmem {
    uint4 w[kFragFwd];
    float bias[kBias];
    float freq[2 * kNF];
};

__device__ __forceinline__ void stage_network(MlpSmem &sm, const uint4 *__restrict__ wf,
                                              const float *__restrict__ theta,
                                              const float *__restrict__ freq)
{
    for (int i = threadIdx.x; i < kFragFwd; i += blockDim.x) sm.w[i] = wf[i];
    for (int i = threadIdx.x; i < kBias; i += blockDim.x)
        sm.bias[i] = i < 4 * kHd ? theta[offB(i / kHd) + i % kHd] : theta[kOffB5 + i - 4 * kHd];
    for (int i = threadIdx.x; i < 2 * kNF; i += blockDim.x) sm.freq[i] = freq[i];
    __syncthreads();
}

__global__ __launch_bounds__(kThreads) void k_mlp_fwd(const uint4 *__restrict__ wf,
                                                      const float *__restrict__ theta,
                                                      const float *__restrict__ freq, int64_t n,
                                                      const float *__restrict__ hin,
                                                      float *__restrict__ yout)
{
    extern __shared__ uint4 s_raw[];
    MlpSmem &sm = *reinterpret_cast<MlpSmem *>(s_raw);
    stage_network(sm, wf, theta, freq);
    const int lane = threadIdx.x % kW, wave = threadIdx.x / kW;
    const int64_t groups = (n + kW - 1) / kW;
    for (int64_t gi = (int64_t)blockIdx.x * (kThreads / kW) + wave; gi < groups;
         gi += (int64_t)gridDim.x * (kThreads / kW)) {
        const int64_t k = gi * kW + lane;
        const bool ok = k < n;
        const float hx = ok ? hin[k] : 0.5f, hy = ok ? hin[n + k] : 0.5f;
        float y[kNO];
        mlp_forward(sm.w, sm.bias, sm.freq, hx, hy, y);
        if (ok)
#pragma unroll
            for (int o = 0; o < kNO; ++o) yout[(int64_t)o * n + k] = y[o];
    }
}

// ---------------------------------------------------------------------------
// Training: forward + backward of 64 samples per wave
// act:  a_0..a_4, unit-major BF16, a_l[u * bn + i]
// dz:   dZ_1..dZ_4 (128 units each) then dY (16), unit-major BF16
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_mlp_train(
    const uint4 *__restrict__ wf, const uint4 *__restrict__ wb, const float *__restrict__ theta,
    const float *__restrict__ freq, const float *__restrict__ samples, int64_t n_samples,
    uint64_t idx_base, uint64_t idx_mult, int32_t n_valid, int32_t bn, uint16_t *__restrict__ act,
    uint16_t *__restrict__ dz, float *__restrict__ loss_part)
{
    __shared__ float s_loss[kThreads / kW];
    __shared__ uint64_t s_mask[kThreads / kW][4][kW];     // relu masks, per wave, layer, lane
    const int lane = threadIdx.x % kW, wave = threadIdx.x / kW, h = lane / 32, n = lane % 32;
    const int32_t i0 = (blockIdx.x * (kThreads / kW) + wave) * kW;    // first batch slot
    const int32_t i = i0 + lane;                                      // the lane's own slot
    const bool valid = i < n_valid;
    int64_t s = 0;
    if (valid) s = (int64_t)((((idx_base + (uint64_t)i) % (uint64_t)n_samples) * idx_mult) % (uint64_t)n_samples);
    float f[20];
#pragma unroll
    for (int e = 0; e < 20; ++e) f[e] = valid ? samples[(int64_t)e * n_samples + s] : 0.0f;
    const float hx = valid ? f[0] : 0.5f, hy = valid ? f[1] : 0.5f;
    float lw = 0.0f;

#pragma unroll 1
    for (int nb = 0; nb < 2; ++nb) {
        const int32_t col = i0 + 32 * nb + n;        // slot of this column
        uint4 B[8];
        features(freq, __shfl(hx, 32 * nb + n), __shfl(hy, 32 * nb + n), B);
        {
            // unit 16 t + 8 h + v: lane part 8 h, uniform part 16 t + v
            uint16_t *lp = act + (int64_t)(8 * h) * bn + col;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const uint32_t w4[4] = {B[t].x, B[t].y, B[t].z, B[t].w};
#pragma unroll
                for (int v = 0; v < 8; ++v)
                    lp[(16 * t + v) * bn] = (uint16_t)(w4[v / 2] >> (16 * (v % 2)));
            }
        }
#pragma unroll 1
        for (int L = 0; L < 4; ++L) {
            uint64_t mk;
            hidden_layer<true>(wf + L * kFragHidden, theta + offB(L), B, mk);
            s_mask[wave][L][lane] = mk;
            // unit 16 t + 8 (v/4) + 4 h + v%4: lane part 4 h, uniform part the rest
            uint16_t *lp = act + ((int64_t)(L + 1) * kHd + 4 * h) * bn + col;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const uint32_t w4[4] = {B[t].x, B[t].y, B[t].z, B[t].w};
#pragma unroll
                for (int v = 0; v < 8; ++v)
                    lp[(16 * t + 8 * (v / 4) + v % 4) * bn] = (uint16_t)(w4[v / 2] >> (16 * (v % 2)));
            }
        }
        float y[kNO];
#pragma unroll
        for (int o = 0; o < kNO; ++o) y[o] = 0.0f;
        head_layer(wf + 4 * kFragHidden, theta + kOffB5, B, nb, y);

        // the owner lanes: loss and d loss / d y of their sample
        const bool owner = h == nb;
        float dy[kNO];
        {
            float pr, pi;
            combine(y, f + 2, pr, pi);
            const bool use = owner && valid;
            const float rr = use ? pr - f[18] : 0.0f, ri = use ? pi - f[19] : 0.0f;
            const float sc = 2.0f / (float)n_valid;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float Dr = f[2 + 2 * k], Di = f[3 + 2 * k];
                dy[2 * k] = sc * (rr * Dr + ri * Di);
                dy[2 * k + 1] = sc * (ri * Dr - rr * Di);
            }
            lw += rr * rr + ri * ri;
            if (owner) {
                uint16_t *dst = dz + (int64_t)4 * kHd * bn;
#pragma unroll
                for (int o = 0; o < kNO; ++o) dst[(int64_t)o * bn + col] = f2bf(dy[o]);
            }
        }
        // dY as the B operand of W5^T: rows 8(v/4) + 4h + v%4 of the column's
        // sample; the owner has them, its partner receives the rows of its half
        uint4 Bd;
        {
            float mine[8], send[8], recv[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const int r0 = 8 * (v / 4) + v % 4;
                mine[v] = h ? dy[r0 + 4] : dy[r0];
                send[v] = h ? dy[r0] : dy[r0 + 4];
            }
#pragma unroll
            for (int v = 0; v < 8; ++v) recv[v] = __shfl_xor(send[v], 32);
            float src[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) src[v] = owner ? mine[v] : recv[v];
            Bd = make_uint4(pack2(src[0], src[1]), pack2(src[2], src[3]), pack2(src[4], src[5]),
                            pack2(src[6], src[7]));
        }
        f32x16 acc[4];
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
            f32x16 z;
#pragma unroll
            for (int r = 0; r < 16; ++r) z[r] = 0.0f;
            acc[ib] = mfma(wb[3 * kFragHidden + ib * kW + lane], Bd, z);
        }
        // dZ_L = dA_L (.) [a_L > 0]; dA_{L-1} = W_L^T dZ_L
#pragma unroll 1
        for (int L = 3; L >= 0; --L) {
            const uint64_t mk = s_mask[wave][L][lane];
            uint16_t *lp = dz + ((int64_t)L * kHd + 4 * h) * bn + col;    // unit drow(mb, r, h)
#pragma unroll
            for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    float o[8];
#pragma unroll
                    for (int v = 0; v < 8; ++v) {
                        const int bit = 16 * mb + 8 * j + v;
                        o[v] = ((mk >> bit) & 1ull) ? acc[mb][8 * j + v] : 0.0f;
                        lp[(32 * mb + 8 * ((8 * j + v) / 4) + v % 4) * bn] = f2bf(o[v]);
                    }
                    B[2 * mb + j] = make_uint4(pack2(o[0], o[1]), pack2(o[2], o[3]), pack2(o[4], o[5]),
                                               pack2(o[6], o[7]));
                }
            if (L == 0) break;
#pragma unroll
            for (int ib = 0; ib < 4; ++ib)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[ib][r] = 0.0f;
            const uint4 *w = wb + (L - 1) * kFragHidden;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
#pragma unroll
                for (int ib = 0; ib < 4; ++ib) acc[ib] = mfma(w[(ib * 8 + t) * kW + lane], B[t], acc[ib]);
                asm volatile("" ::: "memory");
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lw += __shfl_xor(lw, o);
    if (lane == 0) s_loss[wave] = lw;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int w = 0; w < kThreads / kW; ++w) t += s_loss[w];
        loss_part[blockIdx.x] = t;
    }
}

// Weight gradients: dW_l[u][c] = sum_i dZ_l[u][i] a_{l-1}[c][i] over a chunk of
// the batch (one wave per 32 x 32 tile and chunk); bias gradients: sum_i dZ.
// Items per chunk: 64 hidden tiles, 4 head tiles, 5 bias rows.
constexpr int kGradItems = 4 * 16 + 4 + 5;

__global__ __launch_bounds__(kW) void k_mlp_wgrad(const uint16_t *__restrict__ act,
                                                   const uint16_t *__restrict__ dz, int32_t bn,
                                                   int32_t chunk, float *__restrict__ part)
{
    const int lane = threadIdx.x, h = lane / 32, m = lane % 32;
    const int item = blockIdx.x % kGradItems, kc = blockIdx.x / kGradItems;
    const int32_t s0 = kc * chunk, s1 = min(bn, s0 + chunk);
    float *out = part + (int64_t)kc * kNP;
    if (item < 68) {
        int l, ob, ib;
        if (item < 64) { l = item / 16; ob = (item % 16) / 4; ib = item % 4; }
        else { l = 4; ob = 0; ib = item - 64; }
        const uint16_t *dzl = l < 4 ? dz + (int64_t)l * kHd * bn : dz + (int64_t)4 * kHd * bn;
        const uint16_t *al = act + (int64_t)l * kHd * bn;
        const int urow = 32 * ob + m;
        const bool rowok = l < 4 || urow < kNO;
        f32x16 acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
        for (int32_t s = s0; s < s1; s += 16) {
            const uint4 a = rowok ? *reinterpret_cast<const uint4 *>(dzl + (int64_t)urow * bn + s + 8 * h)
                                  : make_uint4(0, 0, 0, 0);
            const uint4 b = *reinterpret_cast<const uint4 *>(al + (int64_t)(32 * ib + m) * bn + s + 8 * h);
            acc = mfma(a, b, acc);
        }
        const int base = l < 4 ? offW(l) : kOffW5;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int u = drow(ob, r, h);
            if (l < 4 || u < kNO) out[base + u * kHd + 32 * ib + m] = acc[r];
        }
    } else {
        const int l = item - 68;
        const int nu = l < 4 ? kHd : kNO;
        const uint16_t *dzl = dz + (int64_t)l * kHd * bn;     // dY follows dZ_4
        for (int u = lane; u < nu; u += kW) {
            float t = 0.0f;
            for (int32_t s = s0; s < s1; ++s) t += bf2f(dzl[(int64_t)u * bn + s]);
            out[(l < 4 ? offB(l) : kOffB5) + u] = t;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_mlp_reduce(const float *__restrict__ part, int32_t nchunk,
                                                         const float *__restrict__ loss_part,
                                                         int32_t nloss, float *__restrict__ grad,
                                                         double *__restrict__ loss_out)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p < kNP) {
        float t = 0.0f;
        for (int k = 0; k < nchunk; ++k) t += part[(int64_t)k * kNP + p];
        grad[p] = t;
    }
    if (p == 0 && loss_out) {
        double t = 0.0;
        for (int k = 0; k < nloss; ++k) t += (double)loss_part[k];
        *loss_out = t;
    }
}

__global__ __launch_bounds__(kThreads) void k_adam(float *__restrict__ theta, float *__restrict__ m,
                                                   float *__restrict__ v, const float *__restrict__ g,
                                                   float lr, float b1, float b2, float eps, float c1,
                                                   float c2)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= kNP) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    theta[p] -= lr * (mp * c1) / (sqrtf(vp * c2) + eps);
}

__global__ __launch_bounds__(kThreads) void k_learn_err(const float *__restrict__ samples, int64_t n,
                                                        const float *__restrict__ y,
                                                        float *__restrict__ err_learn,
                                                        float *__restrict__ err_base)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    float yy[kNO], D[16];
#pragma unroll
    for (int o = 0; o < kNO; ++o) yy[o] = y[(int64_t)o * n + k];
#pragma unroll
    for (int e = 0; e < 16; ++e) D[e] = samples[(int64_t)(2 + e) * n + k];
    float pr, pi;
    combine(yy, D, pr, pi);
    const float Tr = samples[18 * n + k], Ti = samples[19 * n + k], sg = samples[20 * n + k];
    err_learn[k] = sg * sqrtf((pr - Tr) * (pr - Tr) + (pi - Ti) * (pi - Ti));
    err_base[k] = sg * sqrtf(Tr * Tr + Ti * Ti);
}

// The learned path's column table: ray column i's square column
// gxc = floor((i + 1/2) n1x qc / nx) and level-1 column gxc / qc.
__global__ __launch_bounds__(kThreads) void k_learn_cols(DevGeom g, int32_t qc, int2 *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= g.nx) return;
    const int64_t gxc = ((2 * i + 1) * ((int64_t)g.n1x * qc)) / (2 * g.nx);
    out[i] = make_int2((int32_t)gxc, (int32_t)(gxc / qc));
}

// The blended weights at n offsets hin (hx row, hy row) from the table tab
// (output-major: tab[o kLNodes + node]) into yout (16 x n: yout[o n + k]).
__global__ __launch_bounds__(kThreads) void k_ltab_eval(const float *__restrict__ tab, int64_t n,
                                                        const float *__restrict__ hin,
                                                        float *__restrict__ yout)
{
    for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * kThreads) {
        float y[kNO];
        ltab_blend<1, kLNodes>(tab, hin[k], hin[n + k], y);
#pragma unroll
        for (int o = 0; o < kNO; ++o) yout[(int64_t)o * n + k] = y[o];
    }
}

// ---------------------------------------------------------------------------
// Rays with the learned interpolant.  One wave item = 64 consecutive columns
// of kLearnRows rows (a lane takes one column's rows); a persistent workgroup
// of 6 waves keeps the weight table in LDS and walks the band's items.
// ---------------------------------------------------------------------------
constexpr int kL3Threads = 384;

// One nearby lens's term m (d1, d2)/r^2, d = theta - z: m/r^2 is the
// hardware reciprocal estimate times m corrected once (relative error about
// the square of the estimate's, <= 2.2e-15); 1e-300 added to d1^2 leaves any
// r^2 above ~1e-284 unchanged and makes the term of a lens exactly on the ray
// 0 x finite = 0.
__device__ __forceinline__ void near_lens(double t1, double t2, double zx, double zy, double m,
                                          double &n1, double &n2)
{
    const double d1 = t1 - zx, d2 = t2 - zy;
    const double rr = fma(d2, d2, fma(d1, d1, 1e-300));
    const double v = __builtin_amdgcn_rcp(rr);
    const double y = m * v;
    const double w = fma(v, fma(-rr, y, m), y);
    n1 = fma(w, d1, n1);
    n2 = fma(w, d2, n2);
}

// Rays of columns [i0, i1) and rows [j0, j1) in items of 64 columns of one
// row.  CORNER = false: the sheet's analytic part outside the four corner
// cells of the rectangle, whose rays (with a sheet) it leaves out;
// CORNER = true: rays of one of those cells, with the sheet's closed form
// (its logarithms would otherwise set every ray's register budget).
// rays of a lane: kLearnRows consecutive rows of one column
constexpr int kLearnRows = 4;
template <int A, int B>
struct RowSpan {
    static constexpr int first = A, last = B;
};

#define IRS_LEARNED_RAY_ARGS                                                                      \
    DevGeom g, LearnGeom lg, const double *__restrict__ lx, const double *__restrict__ ly,        \
        const double *__restrict__ lm, const int32_t *__restrict__ cell_start,                    \
        const double *__restrict__ corner, int32_t cy0, const float *__restrict__ tab,            \
        const int2 *__restrict__ lcol, int64_t i0,                                                \
        int64_t i1, int64_t j0, int64_t j1, int64_t ray_first, int64_t ray_last, double *a1o,     \
        double *a2o, int64_t *pixo, uint32_t *counts, unsigned long long *landed
template <bool UNIT, bool CORNER>
__device__ __forceinline__ void learned_rays(IRS_LEARNED_RAY_ARGS)
{
    extern __shared__ uint4 s_raw[];
    float *s_tab = reinterpret_cast<float *>(s_raw);          // node-major: [node][16]
    for (int e = threadIdx.x; e < kLNodes * kNO; e += blockDim.x)
        s_tab[e] = tab[(int64_t)(e % kNO) * kLNodes + e / kNO];
    __syncthreads();
    const int lane = threadIdx.x % kW;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kW);   // items are wave-uniform
    constexpr int kWaves = kL3Threads / kW;
    constexpr int R = kLearnRows;
    const int64_t ntx = (i1 - i0 + kW - 1) / kW;
    const int64_t items = (j1 - j0 + R - 1) / R * ntx;
    const int q1 = lg.qc + 1;
    const int64_t nyc = (int64_t)g.n1y * lg.qc;
    auto cell_row = [&](int64_t j) { return (int32_t)(((2 * j + 1) * nyc) / (2 * g.ny) / lg.qc); };
    unsigned long long nland = 0;
    for (int64_t it = (int64_t)blockIdx.x * kWaves + wave; it < items; it += (int64_t)gridDim.x * kWaves) {
        // rows jg .. jg + nr - 1 of one column per lane
        const int64_t jg = j0 + (it / ntx) * R;
        const int nr = (int)min<int64_t>(R, j1 - jg);
        const int64_t i = i0 + (it % ntx) * kW + lane;
        const bool in_col = i < i1;
        // the lane's square column and level-1 column (lanes past the
        // range take its last column)
        const int2 sq = lcol[in_col ? i : i1 - 1];
        const double t1 = ray_x(g, in_col ? i : i1 - 1);
        double t2s[R], n1[R], n2[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            t2s[k] = ray_y(g, jg + min(k, nr - 1));     // rows past the range repeat the last
            n1[k] = 0.0;
            n2[k] = 0.0;
        }
        // nearby lenses, exactly, in a loop the whole wave shares: the lens
        // data come in scalar loads, each lens serves all the lane's rows of
        // one level-1 row; where the wave's columns straddle two level-1
        // columns a lane gives the lenses outside its own 3 x 3 cells mass 0,
        // adding exact zeros
        {
            const int32_t cxl = sq.y;
            // columns grow with the lane: lane 0 has the first, lane 63 the last
            const int32_t cxa = __builtin_amdgcn_readfirstlane(cxl);
            const int32_t cxb = __builtin_amdgcn_readlane(cxl, kW - 1);
            const int32_t cl = cxa > 0 ? cxa - 1 : 0, ch = cxb < g.n1x - 1 ? cxb + 1 : g.n1x - 1;
            const int32_t xl = cxl > 0 ? cxl - 1 : 0, xh = cxl < g.n1x - 1 ? cxl + 1 : g.n1x - 1;
            const bool straddle = cxa != cxb;
            auto pass = [&](int32_t cyr, auto rows) {           // rows: compile-time [k0, k1)
                constexpr int k0 = decltype(rows)::first, k1 = decltype(rows)::last;
                const int32_t yl = cyr > 0 ? cyr - 1 : 0, yh = cyr < g.n1y - 1 ? cyr + 1 : g.n1y - 1;
                for (int32_t row = yl; row <= yh; ++row) {
                    const int32_t pb = cell_start[row * g.n1x + cl];
                    const int32_t pe = cell_start[row * g.n1x + ch + 1];
                    int32_t lpb = pb, lpe = pe;
                    if (straddle) {
                        lpb = cell_start[row * g.n1x + xl];
                        lpe = cell_start[row * g.n1x + xh + 1];
                    }
                    for (int32_t q_ = pb; q_ < pe; ++q_) {
                        double m = UNIT ? 1.0 : lm[q_];
                        if (straddle) m = (q_ >= lpb && q_ < lpe) ? m : 0.0;
                        const double zx = lx[q_], zy = ly[q_];
#pragma unroll
                        for (int k = k0; k < k1; ++k) near_lens(t1, t2s[k], zx, zy, m, n1[k], n2[k]);
                    }
                }
            };
            const int32_t cyA = cell_row(jg), cyB = cell_row(jg + nr - 1);   // wave-uniform
            if (cyA == cyB) {
                pass(cyA, RowSpan<0, R>{});
            } else {                                        // rows sorted: split by cell row
#pragma unroll
                for (int k = 0; k < R; ++k)
                    if (k < nr) {
                        const int32_t cyk = cell_row(jg + k);
                        if (k == 0) pass(cyk, RowSpan<0, 1>{});
                        else if (k == 1) pass(cyk, RowSpan<1, 2>{});
                        else if (k == 2) pass(cyk, RowSpan<2, 3>{});
                        else pass(cyk, RowSpan<3, 4>{});
                    }
            }
        }
        // per row: the square's corners (cached loads) and, when the square
        // row changes (a wave-uniform test), its local data; then each ray's
        // base interpolant, learned correction, pixel and bin
        const int64_t gxc = sq.x, cx = sq.y;
        const int a = (int)(gxc - cx * lg.qc);
        const double X0 = corner_x(g, lg, gxc), X1 = corner_x(g, lg, gxc + 1);
        const float hx = (float)((t1 - X0) / lg.sx);
        float D[16];
        double sig = 0.0;
        int64_t cgy = -1;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (k >= nr) break;                             // wave-uniform
            const int64_t j = jg + k;
            const int64_t gyc = ((2 * j + 1) * nyc) / (2 * g.ny);
            const int64_t cy = gyc / lg.qc;
            const double Y0 = corner_y(g, lg, gyc), Y1 = corner_y(g, lg, gyc + 1);
            double C[4][4];
            load_corners(corner, (cy - cy0) * g.n1x + cx, q1, a, (int)(gyc - cy * lg.qc), C);
            if (gyc != cgy) {                               // wave-uniform
                square_local(C, X0, X1, Y0, Y1, lg, D, sig);
                cgy = gyc;
            }
            const double t2 = t2s[k];
            const int64_t r = j * g.nx + i;
            bool valid = in_col && r >= ray_first && r < ray_last;
            if (!CORNER && g.sheet && corner_cell_l(g, cx, cy)) valid = false;
            int32_t pix = -1;
            if (valid) {
                const double dhy = (t2 - Y0) / lg.sy;
                double Ar, Ai;
                square_base(C, X0, X1, Y0, Y1, t1, t2, (double)hx, dhy, Ar, Ai);
                if (g.sheet) {
                    if constexpr (CORNER) {
                        double I1, I2;
                        sheet_unit(g, t1, t2, I1, I2);
                        const double f = -g.kappa_star / M_PI;
                        Ar += f * I1;
                        Ai -= f * I2;
                    } else {
                        Ar -= g.kappa_star * t1;          // -kappa_* conj(z)
                        Ai += g.kappa_star * t2;
                    }
                }
                float pr, pi;
                ltab_combine<kNO, 1>(s_tab, hx, (float)dhy, D, pr, pi);
                // alpha: the near lenses, the macro term, the base
                // interpolant and the conjugate of the learned correction
                const double a1 = (g.kpg * t1 + n1[k] + Ar) + sig * (double)pr;
                const double a2 = (g.kmg * t2 + n2[k] - Ai) - sig * (double)pi;
                pix = pixel_of(g, t1 - a1, t2 - a2);
                if (!counts) {
                    const int64_t o = r - ray_first;
                    if (a1o) a1o[o] = a1;
                    if (a2o) a2o[o] = a2;
                    if (pixo) pixo[o] = pix;
                }
            }
            if (counts) {
                bin_runs(counts, pix);
                nland += __popcll(__ballot(pix >= 0));
            }
            asm volatile("" ::: "memory");      // keep the next row's corner loads in its row
        }
    }
    if (counts && lane == 0 && nland) landed_add(landed, nland);
}

#define IRS_LEARNED_RAY_PASS                                                                      \
    g, lg, lx, ly, lm, cell_start, corner, cy0, tab, lcol, i0, i1, j0, j1, ray_first, ray_last, a1o, \
        a2o, pixo, counts, landed
// three waves a SIMD: two workgroups of six waves a CU (the table's LDS allows two)
template <bool UNIT>
__global__ __launch_bounds__(kL3Threads, 3) void k_level3_learned(IRS_LEARNED_RAY_ARGS)
{
    learned_rays<UNIT, false>(IRS_LEARNED_RAY_PASS);
}
// the corner cells: fewer waves, no spills
template <bool UNIT>
__global__ __launch_bounds__(kL3Threads) void k_level3_learned_corner(IRS_LEARNED_RAY_ARGS)
{
    learned_rays<UNIT, true>(IRS_LEARNED_RAY_PASS);
}
#undef IRS_LEARNED_RAY_PASS
#undef IRS_LEARNED_RAY_ARGS

int device_cus()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        return 256;
    return n;
}

constexpr size_t kMlpSmem = sizeof(MlpSmem);
constexpr size_t kLTabSmem = sizeof(float) * kLNodes * kNO;

irs_status set_smem_limits()
{
    static bool done = false;
    if (done) return IRS_OK;
    IRS_HIP(hipFuncSetAttribute((const void *)k_mlp_fwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kMlpSmem));
    const void *ray_kernels[4] = {(const void *)k_level3_learned<true>,
                                  (const void *)k_level3_learned_corner<true>,
                                  (const void *)k_level3_learned<false>,
                                  (const void *)k_level3_learned_corner<false>};
    for (const void *f : ray_kernels)
        IRS_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLTabSmem));
    done = true;
    return IRS_OK;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;                         // elements
    ~DevBuf() { dev_free(p); }
    irs_status alloc(size_t count)
    {
        if (dev_alloc(&p, count * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            n = 0;
            set_error("cannot allocate device memory for the learned interpolant");
            return IRS_E_NOMEM;
        }
        n = count;
        return IRS_OK;
    }
};

LearnGeom learn_geom(const irs_plan_s *p, int qc)
{
    LearnGeom lg{};
    lg.qc = qc;
    lg.sx = (p->dg.a2 - p->dg.a1) / (double)((int64_t)p->dg.n1x * qc);
    lg.sy = (p->dg.b2 - p->dg.b1) / (double)((int64_t)p->dg.n1y * qc);
    return lg;
}

int64_t corner_row_bytes(const irs_plan_s *p, int qc)
{
    return (int64_t)p->dg.n1x * (qc + 1) * (qc + 1) * 4 * (int64_t)sizeof(double);
}

// corners of level-1 rows [c0, c1] into dst (expansion first)
irs_status compute_corners(irs_plan_s *p, int qc, int64_t c0, int64_t c1, double *dst)
{
    irs_status st = launch_level2_expand(p, c0, c1);
    if (st != IRS_OK) return st;
    const int P = level2_order(p);
    const int32_t nxb = (p->dg.n1x + kCells - 1) / kCells;
    const unsigned nb = (unsigned)((c1 - c0 + 1) * nxb);
    const LearnGeom lg = learn_geom(p, qc);
    const int32_t nchunk = level2_chunks(p);
#define IRS_LC(U, PP)                                                                              \
    hipLaunchKernelGGL((k_learn_corners<U, PP>), dim3(nb), dim3(kThreads), 0, p->stream, p->dg, lg, \
                       p->d_x, p->d_y, p->d_m, p->d_cell_start, (int32_t)c0, nxb, nchunk,          \
                       p->d_part, dst)
    if (p->unit_mass) {
        if (P == 32) IRS_LC(true, 32);
        else IRS_LC(true, 48);
    } else {
        if (P == 32) IRS_LC(false, 32);
        else IRS_LC(false, 48);
    }
#undef IRS_LC
    IRS_HIP(hipGetLastError());
    return IRS_OK;
}

// samples of level-1 rows [c0, c1]: corners into `corner_tmp`, then samples
irs_status compute_samples(irs_plan_s *p, int qc, int64_t c0, int64_t c1, int per_cell,
                           uint64_t seed, double *corner_tmp, int64_t n_out, float *out)
{
    irs_status st = compute_corners(p, qc, c0, c1, corner_tmp);
    if (st != IRS_OK) return st;
    const int P = level2_order(p);
    const int32_t nxb = (p->dg.n1x + kCells - 1) / kCells;
    const unsigned nb = (unsigned)((c1 - c0 + 1) * nxb);
    const LearnGeom lg = learn_geom(p, qc);
    const int32_t nchunk = level2_chunks(p);
#define IRS_LS(U, PP)                                                                              \
    hipLaunchKernelGGL((k_learn_samples<U, PP>), dim3(nb), dim3(kThreads), 0, p->stream, p->dg, lg, \
                       p->d_x, p->d_y, p->d_m, p->d_cell_start, (int32_t)c0, nxb, nchunk,          \
                       p->d_part, corner_tmp, per_cell, seed, n_out, out)
    if (p->unit_mass) {
        if (P == 32) IRS_LS(true, 32);
        else IRS_LS(true, 48);
    } else {
        if (P == 32) IRS_LS(false, 32);
        else IRS_LS(false, 48);
    }
#undef IRS_LS
    IRS_HIP(hipGetLastError());
    return IRS_OK;
}

irs_status check_learned_plan(const irs_plan_s *p, int qc, const char *who)
{
    if (!p) {
        set_error(std::string(who) + ": NULL plan");
        return IRS_E_INVALID;
    }
    if (p->params.method != IRS_LEARNED) {
        set_error(std::string(who) + ": the plan's method is not IRS_LEARNED");
        return IRS_E_INVALID;
    }
    if (level2_order(p) <= 0) {
        set_error(std::string(who) + ": IRS_LEVEL2_PAPER plans have no per-cell expansion");
        return IRS_E_UNSUPPORTED;
    }
    if (qc < 1 || qc > 32) {
        set_error(std::string(who) + ": coarse must be in 1..32");
        return IRS_E_INVALID;
    }
    if ((int64_t)p->dg.n1x * qc >= INT32_MAX || (int64_t)p->dg.n1y * qc >= INT32_MAX) {
        set_error(std::string(who) + ": too many squares across the map for 32-bit indices");
        return IRS_E_UNSUPPORTED;
    }
    return IRS_OK;
}

// samples from `rows` level-1 rows centred in `rows` equal slices of the map,
// shifted by `phase` of a slice
std::vector<int64_t> sample_rows(const irs_plan_s *p, int rows, double phase)
{
    std::vector<int64_t> out;
    const int64_t n1y = p->dg.n1y;
    rows = (int)std::max<int64_t>(1, std::min<int64_t>(rows, n1y));
    for (int k = 0; k < rows; ++k) {
        int64_t r = (int64_t)std::floor(((double)k + phase) * (double)n1y / (double)rows);
        r = std::min<int64_t>(n1y - 1, std::max<int64_t>(0, r));
        if (out.empty() || out.back() != r) out.push_back(r);
    }
    return out;
}

// samples for a list of rows (one row per launch), per_cell each
irs_status gather_samples(irs_plan_s *p, int qc, const std::vector<int64_t> &rows, int per_cell,
                          uint64_t seed, float *out, int64_t n_total)
{
    DevBuf<double> ctmp;
    irs_status st = ctmp.alloc((size_t)corner_row_bytes(p, qc) / sizeof(double));
    if (st != IRS_OK) return st;
    DevBuf<float> tmp;
    const int64_t per_row = (int64_t)p->dg.n1x * per_cell;
    st = tmp.alloc((size_t)per_row * kNFld);
    if (st != IRS_OK) return st;
    int64_t off = 0;
    for (int64_t r : rows) {
        st = compute_samples(p, qc, r, r, per_cell, seed, ctmp.p, per_row, tmp.p);
        if (st != IRS_OK) return st;
        for (int e = 0; e < kNFld; ++e)
            IRS_HIP(hipMemcpyAsync(out + (int64_t)e * n_total + off, tmp.p + (int64_t)e * per_row,
                                   sizeof(float) * per_row, hipMemcpyDeviceToDevice, p->stream));
        off += per_row;
    }
    return IRS_OK;
}

// host He initialisation from a splitmix64 stream (Box-Muller normals)
void init_params(uint64_t seed, std::vector<float> &th)
{
    th.assign(kNP, 0.0f);
    uint64_t state = seed * 0x9E3779B97F4A7C15ull + 0x1234567ull;
    auto next = [&state]() {
        uint64_t z = (state += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return (double)((z ^ (z >> 31)) >> 11) * (1.0 / 9007199254740992.0);
    };
    auto normal = [&]() {
        const double u1 = std::max(next(), 1e-300), u2 = next();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    };
    for (int l = 0; l < 4; ++l)
        for (int k = 0; k < kHd * kHd; ++k) th[offW(l) + k] = (float)(normal() * std::sqrt(2.0 / kHd));
    for (int k = 0; k < kNO * kHd; ++k) th[kOffW5 + k] = (float)(normal() * 0.01);
}

irs_status upload_network(irs_plan_s *p, const float *freqs, const float *theta)
{
    if (!p->d_theta) IRS_HIP(dev_alloc(&p->d_theta, sizeof(float) * kNP));
    if (!p->d_freqs) IRS_HIP(dev_alloc(&p->d_freqs, sizeof(float) * 2 * kNF));
    if (!p->d_wfwd) IRS_HIP(dev_alloc(&p->d_wfwd, sizeof(uint4) * kFragFwd));
    IRS_HIP(hipMemcpyAsync(p->d_theta, theta, sizeof(float) * kNP, hipMemcpyHostToDevice, p->stream));
    IRS_HIP(hipMemcpyAsync(p->d_freqs, freqs, sizeof(float) * 2 * kNF, hipMemcpyHostToDevice, p->stream));
    const int64_t ne = (int64_t)kFragFwd * 8;
    hipLaunchKernelGGL(k_mlp_pack, dim3((unsigned)((ne + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       p->stream, p->d_theta, (uint16_t *)p->d_wfwd, (uint16_t *)nullptr);
    IRS_HIP(hipGetLastError());
    return IRS_OK;
}

irs_status launch_mlp_fwd(hipStream_t s, const void *wf, const float *theta, const float *freq,
                          int64_t n, const float *h, float *y)
{
    irs_status st = set_smem_limits();
    if (st != IRS_OK) return st;
    const int64_t groups = (n + kW - 1) / kW;
    const int64_t want = (groups + kThreads / kW - 1) / (kThreads / kW);
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, device_cus()));
    hipLaunchKernelGGL(k_mlp_fwd, dim3(nb), dim3(kThreads), kMlpSmem, s, (const uint4 *)wf, theta,
                       freq, n, h, y);
    IRS_HIP(hipGetLastError());
    return IRS_OK;
}

// the plan's weight table from its current network (on its stream, waited for)
irs_status build_table(irs_plan_s *p)
{
    if (!p->d_ltab) IRS_HIP(dev_alloc(&p->d_ltab, sizeof(float) * kNO * kLNodes));
    std::vector<float> h(2 * kLNodes);
    for (int b = 0; b <= kLTab; ++b)
        for (int a = 0; a <= kLTab; ++a) {
            h[b * (kLTab + 1) + a] = (float)a / (float)kLTab;             // exact: kLTab = 2^5
            h[kLNodes + b * (kLTab + 1) + a] = (float)b / (float)kLTab;
        }
    DevBuf<float> dh;
    irs_status st = dh.alloc(h.size());
    if (st != IRS_OK) return st;
    IRS_HIP(hipMemcpyAsync(dh.p, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, p->stream));
    if ((st = launch_mlp_fwd(p->stream, p->d_wfwd, p->d_theta, p->d_freqs, kLNodes, dh.p,
                             p->d_ltab)) != IRS_OK)
        return st;
    IRS_HIP(hipStreamSynchronize(p->stream));             // before dh is freed
    return IRS_OK;
}

irs_status launch_ltab_eval(hipStream_t s, const float *tab, int64_t n, const float *h, float *y)
{
    const int64_t want = (n + kThreads - 1) / kThreads;
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, 64 * device_cus()));
    hipLaunchKernelGGL(k_ltab_eval, dim3(nb), dim3(kThreads), 0, s, tab, n, h, y);
    IRS_HIP(hipGetLastError());
    return IRS_OK;
}

double quantile(std::vector<float> v, double q)
{
    if (v.empty()) return 0.0;
    const size_t k = std::min(v.size() - 1, (size_t)std::floor(q * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + (long)k, v.end());
    return v[k];
}

// tabulate the plan's network and validate the weights the rays will take
// (the table's) on n_val samples from rows between the training rows; fills
// the report's validation fields and the decision
irs_status validate(irs_plan_s *p, const irs_learn_params &lp, irs_learn_report &rep)
{
    const int qc = p->learn_qc;
    irs_status st0 = build_table(p);
    if (st0 != IRS_OK) return st0;
    const std::vector<int64_t> rows = sample_rows(p, std::max(1, lp.train_rows), 0.5 + 0.25);
    const int64_t per_row_cells = p->dg.n1x;
    const int per_cell = (int)std::max<int64_t>(
        1, (lp.n_val + (int64_t)rows.size() * per_row_cells - 1) / ((int64_t)rows.size() * per_row_cells));
    const int64_t n = (int64_t)rows.size() * per_row_cells * per_cell;
    auto t0 = std::chrono::steady_clock::now();
    DevBuf<float> smp, y, el, eb;
    irs_status st = smp.alloc((size_t)n * kNFld);
    if (st == IRS_OK) st = y.alloc((size_t)n * kNO);
    if (st == IRS_OK) st = el.alloc((size_t)n);
    if (st == IRS_OK) st = eb.alloc((size_t)n);
    if (st != IRS_OK) return st;
    st = gather_samples(p, qc, rows, per_cell, lp.seed ^ 0x5a5a5a5aull, smp.p, n);
    if (st != IRS_OK) return st;
    st = launch_ltab_eval(p->stream, p->d_ltab, n, smp.p, y.p);
    if (st != IRS_OK) return st;
    hipLaunchKernelGGL(k_learn_err, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       p->stream, smp.p, n, y.p, el.p, eb.p);
    IRS_HIP(hipGetLastError());
    std::vector<float> hl(n), hb(n);
    IRS_HIP(hipMemcpyAsync(hl.data(), el.p, sizeof(float) * n, hipMemcpyDeviceToHost, p->stream));
    IRS_HIP(hipMemcpyAsync(hb.data(), eb.p, sizeof(float) * n, hipMemcpyDeviceToHost, p->stream));
    IRS_HIP(hipStreamSynchronize(p->stream));
    double sl = 0.0, sb = 0.0, ml = 0.0, mb = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        sl += hl[k];
        sb += hb[k];
        ml = std::max(ml, (double)hl[k]);
        mb = std::max(mb, (double)hb[k]);
    }
    rep.n_val = n;
    rep.val_mean_abs = sl / (double)n;
    rep.base_mean_abs = sb / (double)n;
    rep.val_max_abs = ml;
    rep.base_max_abs = mb;
    rep.val_p9999_abs = quantile(hl, 0.9999);
    rep.base_p9999_abs = quantile(hb, 0.9999);
    const double dpix = p->geo.info.dpix;
    rep.tol_mean = lp.tol_mean > 0.0 ? lp.tol_mean : 2.5e-5 * dpix;
    rep.tol_p9999 = lp.tol_p9999 > 0.0 ? lp.tol_p9999 : 2.5e-3 * dpix;
    rep.fallback = (rep.val_mean_abs > rep.tol_mean || rep.val_p9999_abs > rep.tol_p9999) ? 1 : 0;
    rep.coarse = qc;
    rep.corner_bytes_per_row = corner_row_bytes(p, qc);
    rep.coef_bytes_per_row = (int64_t)p->dg.n1x * p->dg.q * p->dg.q * 10 * (int64_t)sizeof(double);
    p->learn_ok = rep.fallback == 0;
    p->corner_c0 = -1;
    p->corner_c1 = -2;
    rep.ms_validate = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return IRS_OK;
}

irs_status check_params(const irs_learn_params &lp, bool training)
{
    if (lp.n_val < 1 || lp.train_rows < 1 ||
        (training && (lp.n_samples < 256 || lp.batch < 256 || lp.batch % 256 != 0 || lp.steps < 0 ||
                      !(lp.lr >= 0.0f) || !(lp.beta1 >= 0.0f && lp.beta1 < 1.0f) ||
                      !(lp.beta2 >= 0.0f && lp.beta2 < 1.0f) || !(lp.adam_eps > 0.0f)))) {
        set_error("irs_learn: training settings out of range");
        return IRS_E_INVALID;
    }
    return IRS_OK;
}

// gradient of the loss over n records (device) for parameters already packed
// into wf/wb; fills grad (device) and loss (device, one double)
struct TrainBufs {
    DevBuf<uint16_t> act, dz;
    DevBuf<float> part, loss_part;
    int32_t bn = 0, nchunk = 0;
    irs_status alloc(int32_t batch)
    {
        bn = batch;
        const int32_t chunk = 1024;
        nchunk = (bn + chunk - 1) / chunk;
        irs_status st = act.alloc((size_t)5 * kHd * bn);
        if (st == IRS_OK) st = dz.alloc((size_t)(4 * kHd + kNO) * bn);
        if (st == IRS_OK) st = part.alloc((size_t)nchunk * kNP);
        if (st == IRS_OK) st = loss_part.alloc((size_t)bn / kThreads + 1);
        return st;
    }
};

// The furthest element each training kernel indexes, against the buffers:
// k_mlp_train writes act[(5 kHd) bn], dz[(4 kHd + kNO) bn] and loss_part[nbt]
// for slots up to nbt kThreads (so bn must be a multiple of kThreads);
// k_mlp_wgrad reads slots [kc chunk16, min(bn, kc chunk16 + chunk16)) in
// steps of 16 and writes part[nchunk kNP]; k_mlp_reduce reads what they wrote.
bool train_extents_ok(const TrainBufs &tb, int32_t n_valid)
{
    const int64_t nbt = (tb.bn + kThreads - 1) / kThreads;
    const int32_t chunk = (tb.bn + tb.nchunk - 1) / tb.nchunk;
    const int64_t chunk16 = (chunk + 15) / 16 * 16;
    return tb.bn > 0 && tb.bn % kThreads == 0 && n_valid >= 0 && n_valid <= tb.bn &&
           nbt * kThreads == tb.bn && tb.act.n >= (size_t)5 * kHd * tb.bn &&
           tb.dz.n >= (size_t)(4 * kHd + kNO) * tb.bn && tb.loss_part.n >= (size_t)nbt &&
           tb.part.n >= (size_t)tb.nchunk * kNP && chunk16 % 16 == 0 &&
           (int64_t)tb.nchunk * chunk16 >= tb.bn && tb.bn % 16 == 0;
}

irs_status grad_step(hipStream_t s, TrainBufs &tb, const void *wf, const void *wb, const float *theta,
                     const float *freq, const float *samples, int64_t n_samples, uint64_t base,
                     uint64_t mult, int32_t n_valid, float *grad, double *loss)
{
    if (!train_extents_ok(tb, n_valid)) {
        set_error("internal: training buffers smaller than the kernels index");
        return IRS_E_INVALID;
    }
    const unsigned nbt = (unsigned)((tb.bn + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_mlp_train, dim3(nbt), dim3(kThreads), 0, s, (const uint4 *)wf,
                       (const uint4 *)wb, theta, freq, samples, n_samples, base, mult, n_valid, tb.bn,
                       tb.act.p, tb.dz.p, tb.loss_part.p);
    const int32_t chunk = (tb.bn + tb.nchunk - 1) / tb.nchunk;
    const int32_t chunk16 = (chunk + 15) / 16 * 16;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((unsigned)(kGradItems * tb.nchunk)), dim3(kW), 0, s, tb.act.p,
                       tb.dz.p, tb.bn, chunk16, tb.part.p);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)((kNP + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       s, tb.part.p, tb.nchunk, tb.loss_part.p, (int32_t)nbt, grad, loss);
    IRS_HIP(hipGetLastError());
    return IRS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Entry points used by the C ABI
// ---------------------------------------------------------------------------
void learn_release(irs_plan_s *p)
{
    dev_free(p->d_theta);
    dev_free(p->d_freqs);
    dev_free(p->d_wfwd);
    dev_free(p->d_ltab);
    dev_free(p->d_lcol);
    dev_free(p->d_corner);
    p->d_theta = p->d_freqs = nullptr;
    p->d_wfwd = nullptr;
    p->d_ltab = nullptr;
    p->d_lcol = nullptr;
    p->lcol_qc = 0;
    p->d_corner = nullptr;
}

irs_status launch_learned(irs_plan_s *p, const RaySel &sel)
{
    if (p->learn_qc == 0) {
        set_error("IRS_LEARNED plan has no network: call irs_learn or irs_learn_set first");
        return IRS_E_INVALID;
    }
    if (!p->learn_ok) return launch_interp(p, sel);        // validated fallback
    if (sel.row1 <= sel.row0) return IRS_OK;
    irs_status st = set_smem_limits();
    if (st != IRS_OK) return st;
    const DevGeom &g = p->dg;
    const int qc = p->learn_qc;
    const LearnGeom lg = learn_geom(p, qc);
    const int64_t nyc = (int64_t)g.n1y * qc;
    auto cell_row = [&](int64_t j) { return ((2 * j + 1) * nyc) / (2 * g.ny) / qc; };
    const int64_t cyA = cell_row(sel.row0), cyB = cell_row(sel.row1 - 1);
    // band height: the corner table is small; the partial expansions bound it
    const int P = level2_order(p);
    const int64_t part_row = (int64_t)g.n1x * level2_chunks(p) * P * 2 * (int64_t)sizeof(double);
    const int64_t band = std::max<int64_t>(1, std::min<int64_t>(g.n1y, ((int64_t)1 << 30) / part_row));
    if (p->corner_rows_cap < band) {
        dev_free(p->d_corner);
        p->d_corner = nullptr;
        p->corner_rows_cap = 0;
        p->corner_c0 = -1;
        p->corner_c1 = -2;
        IRS_HIP(dev_alloc(&p->d_corner, (size_t)(band * corner_row_bytes(p, qc))));
        p->corner_rows_cap = band;
    }
    if (!p->d_lcol || p->lcol_qc != qc) {                 // the column table, per coarse grid
        dev_free(p->d_lcol);
        p->d_lcol = nullptr;
        p->lcol_qc = 0;
        IRS_HIP(dev_alloc(&p->d_lcol, sizeof(int2) * (size_t)g.nx));
        hipLaunchKernelGGL(k_learn_cols, dim3((unsigned)((g.nx + kThreads - 1) / kThreads)),
                           dim3(kThreads), 0, p->stream, g, (int32_t)qc, (int2 *)p->d_lcol);
        IRS_HIP(hipGetLastError());
        p->lcol_qc = qc;
    }
    CallStats *cs = sel.stats;
    const int ncu = device_cus();
    int per_cu = 0;                         // resident workgroups per CU (the table in LDS)
    if (p->unit_mass)
        IRS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_level3_learned<true>,
                                                             kL3Threads, kLTabSmem));
    else
        IRS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_level3_learned<false>,
                                                             kL3Threads, kLTabSmem));
    per_cu = std::max(1, per_cu);
    for (int64_t c0 = cyA; c0 <= cyB; c0 += p->corner_rows_cap) {
        const int64_t c1 = std::min(cyB, c0 + p->corner_rows_cap - 1);
        if (!(p->corner_c0 <= c0 && c1 <= p->corner_c1)) {
            if (cs) {
                st = cs->begin(p->stream, 0);
                if (st != IRS_OK) return st;
                cs->n_level2++;
                cs->level2_points += (c1 - c0 + 1) * g.n1x * (qc + 1) * (qc + 1);
            }
            st = compute_corners(p, qc, c0, c1, p->d_corner);
            if (st != IRS_OK) return st;
            if (cs && (st = cs->end(p->stream)) != IRS_OK) return st;
            p->corner_c0 = c0;
            p->corner_c1 = c1;
        }
        // rays of these cell rows (cell_row is non-decreasing in j)
        auto first_row = [&](int64_t cr) {
            int64_t lo = sel.row0, hi = sel.row1;
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (cell_row(mid) >= cr) hi = mid;
                else lo = mid + 1;
            }
            return lo;
        };
        const int64_t jA = first_row(c0), jB = first_row(c1 + 1);
        if (jB <= jA) continue;
        if (cs) {
            st = cs->begin(p->stream, 1);
            if (st != IRS_OK) return st;
            cs->n_rays++;
        }
        // rays of columns [i0, i1), rows [ja, jb): the main kernel, or one
        // corner cell's
        auto launch = [&](bool corner_cell, int64_t i0, int64_t i1, int64_t ja, int64_t jb) {
            const int64_t items = (jb - ja + kLearnRows - 1) / kLearnRows * ((i1 - i0 + kW - 1) / kW);
            const unsigned nb = (unsigned)std::max<int64_t>(
                1, std::min<int64_t>((int64_t)per_cu * ncu, (items + kL3Threads / kW - 1) / (kL3Threads / kW)));
#define IRS_L3L(K)                                                                                 \
    hipLaunchKernelGGL(K, dim3(nb), dim3(kL3Threads), kLTabSmem, p->stream, g, lg, p->d_x, p->d_y,  \
                       p->d_m, p->d_cell_start, p->d_corner, (int32_t)p->corner_c0, p->d_ltab,      \
                       (const int2 *)p->d_lcol, i0,                                                \
                       i1, ja, jb, sel.ray_first, sel.ray_last, sel.alpha1, sel.alpha2, sel.pixel, \
                       sel.counts, sel.landed)
            if (p->unit_mass) {
                if (corner_cell) IRS_L3L(k_level3_learned_corner<true>);
                else IRS_L3L(k_level3_learned<true>);
            } else {
                if (corner_cell) IRS_L3L(k_level3_learned_corner<false>);
                else IRS_L3L(k_level3_learned<false>);
            }
#undef IRS_L3L
        };
        launch(false, 0, g.nx, jA, jB);
        if (g.sheet) {
            // the rectangle's corner cells (distinct ones) that meet these rows
            const int64_t cxs[2] = {0, g.n1x - 1}, cys[2] = {0, g.n1y - 1};
            for (int ky = 0; ky < (g.n1y > 1 ? 2 : 1); ++ky)
                for (int kx = 0; kx < (g.n1x > 1 ? 2 : 1); ++kx) {
                    int64_t ia, ib, ra, rb;
                    level1_span(p->geo.info, 0, cxs[kx], ia, ib);
                    level1_span(p->geo.info, 1, cys[ky], ra, rb);
                    ra = std::max(ra, jA);
                    rb = std::min(rb, jB);
                    if (ia < ib && ra < rb) launch(true, ia, ib, ra, rb);
                }
        }
        IRS_HIP(hipGetLastError());
        if (cs && (st = cs->end(p->stream)) != IRS_OK) return st;
    }
    return IRS_OK;
}

}  // namespace irs

using namespace irs;

extern "C" {

irs_status irs_learn_defaults(irs_learn_params *out)
{
    if (!out) {
        set_error("irs_learn_defaults: NULL argument");
        return IRS_E_INVALID;
    }
    irs_learn_params d{};
    d.coarse = 16;
    d.train_rows = 8;
    d.n_samples = 2000000;
    d.n_val = 200000;
    d.batch = 8192;
    d.steps = 6000;
    d.lr = 2e-3f;
    d.lr_final = 2e-5f;
    d.beta1 = 0.9f;
    d.beta2 = 0.999f;
    d.adam_eps = 1e-8f;
    d.seed = 12345;
    d.tol_mean = 0.0;
    d.tol_p9999 = 0.0;
    *out = d;
    return IRS_OK;
}

irs_status irs_learn(irs_plan_t p, const irs_learn_params *lpp, const float *freqs,
                     const float *theta0, irs_learn_report *report)
{
    irs_learn_params lp;
    if (lpp) lp = *lpp;
    else irs_learn_defaults(&lp);
    irs_status st = check_learned_plan(p, lp.coarse, "irs_learn");
    if (st != IRS_OK) return st;
    if (!freqs) {
        set_error("irs_learn: NULL frequencies");
        return IRS_E_INVALID;
    }
    if ((st = check_params(lp, true)) != IRS_OK) return st;
    irs_learn_report rep{};
    const hipStream_t s = p->stream;
    const int qc = lp.coarse;

    // 1. exact samples
    auto t0 = std::chrono::steady_clock::now();
    const std::vector<int64_t> rows = sample_rows(p, lp.train_rows, 0.5);
    const int64_t cells = (int64_t)rows.size() * p->dg.n1x;
    const int per_cell = (int)std::max<int64_t>(1, (lp.n_samples + cells - 1) / cells);
    const int64_t n = cells * per_cell;
    DevBuf<float> smp;
    if ((st = smp.alloc((size_t)n * kNFld)) != IRS_OK) return st;
    if ((st = gather_samples(p, qc, rows, per_cell, lp.seed, smp.p, n)) != IRS_OK) return st;
    IRS_HIP(hipStreamSynchronize(s));
    rep.n_samples = n;
    rep.ms_samples = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();

    // 2. training
    t0 = std::chrono::steady_clock::now();
    std::vector<float> th;
    if (theta0) th.assign(theta0, theta0 + kNP);
    else init_params(lp.seed, th);
    p->learn_qc = qc;
    p->learn_ok = false;
    if ((st = upload_network(p, freqs, th.data())) != IRS_OK) return st;
    DevBuf<uint16_t> wb;
    DevBuf<float> grad, mom, var;
    DevBuf<double> losses;
    TrainBufs tb;
    if ((st = wb.alloc((size_t)kFragBwd * 8)) != IRS_OK) return st;
    if ((st = grad.alloc(kNP)) != IRS_OK || (st = mom.alloc(kNP)) != IRS_OK ||
        (st = var.alloc(kNP)) != IRS_OK)
        return st;
    if ((st = losses.alloc((size_t)std::max(1, lp.steps))) != IRS_OK) return st;
    if ((st = tb.alloc(lp.batch)) != IRS_OK) return st;
    IRS_HIP(hipMemsetAsync(mom.p, 0, sizeof(float) * kNP, s));
    IRS_HIP(hipMemsetAsync(var.p, 0, sizeof(float) * kNP, s));
    const int64_t ne = (int64_t)(kFragFwd + kFragBwd) * 8;
    const unsigned nbp = (unsigned)((ne + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_mlp_pack, dim3(nbp), dim3(kThreads), 0, s, p->d_theta, (uint16_t *)p->d_wfwd, wb.p);
    // a multiplier coprime to n scatters consecutive batch slots over the cells
    uint64_t mult = 2654435761ull % (uint64_t)n;
    auto gcd = [](uint64_t a, uint64_t b) { while (b) { const uint64_t t = a % b; a = b; b = t; } return a; };
    while (mult < 2 || gcd(mult, (uint64_t)n) != 1) mult = (mult + 1) % (uint64_t)n;
    const unsigned nba = (unsigned)((kNP + kThreads - 1) / kThreads);
    double b1t = 1.0, b2t = 1.0;
    for (int step = 0; step < lp.steps; ++step) {
        st = grad_step(s, tb, p->d_wfwd, wb.p, p->d_theta, p->d_freqs, smp.p, n,
                       (uint64_t)step * (uint64_t)lp.batch, mult, lp.batch, grad.p, losses.p + step);
        if (st != IRS_OK) return st;
        b1t *= lp.beta1;
        b2t *= lp.beta2;
        const double frac = lp.steps > 1 ? (double)step / (double)(lp.steps - 1) : 1.0;
        const float lr = (float)(lp.lr_final + 0.5 * (lp.lr - lp.lr_final) * (1.0 + std::cos(M_PI * frac)));
        hipLaunchKernelGGL(k_adam, dim3(nba), dim3(kThreads), 0, s, p->d_theta, mom.p, var.p, grad.p, lr,
                           lp.beta1, lp.beta2, lp.adam_eps, (float)(1.0 / (1.0 - b1t)),
                           (float)(1.0 / (1.0 - b2t)));
        hipLaunchKernelGGL(k_mlp_pack, dim3(nbp), dim3(kThreads), 0, s, p->d_theta, (uint16_t *)p->d_wfwd,
                           wb.p);
        IRS_HIP(hipGetLastError());
    }
    std::vector<double> hl((size_t)std::max(1, lp.steps), 0.0);
    if (lp.steps > 0)
        IRS_HIP(hipMemcpyAsync(hl.data(), losses.p, sizeof(double) * lp.steps, hipMemcpyDeviceToHost, s));
    IRS_HIP(hipStreamSynchronize(s));
    if (lp.steps > 0) {
        const int k = std::max(1, lp.steps / 20);
        double a = 0.0, b = 0.0;
        for (int i = 0; i < k; ++i) {
            a += hl[i] / lp.batch;
            b += hl[lp.steps - 1 - i] / lp.batch;
        }
        rep.loss_first = a / k;
        rep.loss_last = b / k;
    }
    rep.steps = lp.steps;
    rep.ms_train = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();

    // 3. validation and the decision
    if ((st = validate(p, lp, rep)) != IRS_OK) return st;
    if (report) *report = rep;
    set_error("");
    return IRS_OK;
}

irs_status irs_learn_set(irs_plan_t p, const irs_learn_params *lpp, const float *freqs,
                         const float *theta, irs_learn_report *report)
{
    irs_learn_params lp;
    if (lpp) lp = *lpp;
    else irs_learn_defaults(&lp);
    irs_status st = check_learned_plan(p, lp.coarse, "irs_learn_set");
    if (st != IRS_OK) return st;
    if (!freqs || !theta) {
        set_error("irs_learn_set: NULL frequencies or parameters");
        return IRS_E_INVALID;
    }
    if ((st = check_params(lp, false)) != IRS_OK) return st;
    p->learn_qc = lp.coarse;
    p->learn_ok = false;
    if ((st = upload_network(p, freqs, theta)) != IRS_OK) return st;
    irs_learn_report rep{};
    if ((st = validate(p, lp, rep)) != IRS_OK) return st;
    if (report) *report = rep;
    set_error("");
    return IRS_OK;
}

irs_status irs_learn_get(irs_plan_t p, float *freqs, float *theta, int32_t *coarse)
{
    if (!p || p->learn_qc == 0 || !p->d_theta) {
        set_error("irs_learn_get: the plan has no network");
        return IRS_E_INVALID;
    }
    if (freqs) IRS_HIP(hipMemcpy(freqs, p->d_freqs, sizeof(float) * 2 * kNF, hipMemcpyDeviceToHost));
    if (theta) IRS_HIP(hipMemcpy(theta, p->d_theta, sizeof(float) * kNP, hipMemcpyDeviceToHost));
    if (coarse) *coarse = p->learn_qc;
    return IRS_OK;
}

irs_status irs_learn_corners(irs_plan_t p, int32_t coarse, int64_t row0, int64_t nrows, double *out)
{
    irs_status st = check_learned_plan(p, coarse, "irs_learn_corners");
    if (st == IRS_E_INVALID && p && p->params.method != IRS_LEARNED && p->params.method == IRS_INTERP &&
        level2_order(p) > 0 && coarse >= 1 && coarse <= 32)
        st = IRS_OK;                          // interpolation plans may be inspected too
    if (st != IRS_OK) return st;
    if (!out || row0 < 0 || nrows < 1 || row0 + nrows > p->dg.n1y) {
        set_error("irs_learn_corners: NULL output or rows outside [0, n1y)");
        return IRS_E_INVALID;
    }
    DevBuf<double> d;
    const size_t bytes = (size_t)(nrows * corner_row_bytes(p, coarse));
    if ((st = d.alloc(bytes / sizeof(double))) != IRS_OK) return st;
    if ((st = compute_corners(p, coarse, row0, row0 + nrows - 1, d.p)) != IRS_OK) return st;
    IRS_HIP(hipMemcpyAsync(out, d.p, bytes, hipMemcpyDeviceToHost, p->stream));
    IRS_HIP(hipStreamSynchronize(p->stream));
    return IRS_OK;
}

irs_status irs_learn_samples(irs_plan_t p, int32_t coarse, int64_t row0, int64_t nrows,
                             int32_t per_cell, uint64_t seed, float *out)
{
    irs_status st = check_learned_plan(p, coarse, "irs_learn_samples");
    if (st != IRS_OK) return st;
    if (!out || row0 < 0 || nrows < 1 || row0 + nrows > p->dg.n1y || per_cell < 1) {
        set_error("irs_learn_samples: NULL output, rows outside [0, n1y) or per_cell < 1");
        return IRS_E_INVALID;
    }
    std::vector<int64_t> rows;
    for (int64_t r = row0; r < row0 + nrows; ++r) rows.push_back(r);
    const int64_t n = nrows * p->dg.n1x * per_cell;
    if ((st = gather_samples(p, coarse, rows, per_cell, seed, out, n)) != IRS_OK) return st;
    IRS_HIP(hipStreamSynchronize(p->stream));
    return IRS_OK;
}

irs_status irs_learn_weights(irs_plan_t p, int64_t n, const float *h, float *y)
{
    if (!p || n < 0 || (n > 0 && (!h || !y))) {
        set_error("irs_learn_weights: NULL argument or n < 0");
        return IRS_E_INVALID;
    }
    if (p->learn_qc == 0 || !p->d_ltab) {
        set_error("irs_learn_weights: the plan has no network");
        return IRS_E_INVALID;
    }
    if (n == 0) return IRS_OK;
    irs_status st = launch_ltab_eval(p->stream, p->d_ltab, n, h, y);
    if (st != IRS_OK) return st;
    IRS_HIP(hipStreamSynchronize(p->stream));
    return IRS_OK;
}

irs_status irs_mlp_forward(int64_t n, const float *freqs, const float *theta, const float *h, float *y,
                           void *hip_stream)
{
    if (n < 0 || !freqs || !theta || (n > 0 && (!h || !y))) {
        set_error("irs_mlp_forward: NULL argument or n < 0");
        return IRS_E_INVALID;
    }
    if (n == 0) return IRS_OK;
    const hipStream_t s = (hipStream_t)hip_stream;
    DevBuf<float> dth, dfr;
    DevBuf<uint4> wf;
    irs_status st;
    if ((st = dth.alloc(kNP)) != IRS_OK || (st = dfr.alloc(2 * kNF)) != IRS_OK ||
        (st = wf.alloc(kFragFwd)) != IRS_OK)
        return st;
    IRS_HIP(hipMemcpyAsync(dth.p, theta, sizeof(float) * kNP, hipMemcpyHostToDevice, s));
    IRS_HIP(hipMemcpyAsync(dfr.p, freqs, sizeof(float) * 2 * kNF, hipMemcpyHostToDevice, s));
    const int64_t ne = (int64_t)kFragFwd * 8;
    hipLaunchKernelGGL(k_mlp_pack, dim3((unsigned)((ne + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       dth.p, (uint16_t *)wf.p, (uint16_t *)nullptr);
    IRS_HIP(hipGetLastError());
    if ((st = launch_mlp_fwd(s, wf.p, dth.p, dfr.p, n, h, y)) != IRS_OK) return st;
    IRS_HIP(hipStreamSynchronize(s));
    return IRS_OK;
}

irs_status irs_mlp_loss_grad(int64_t n, const float *freqs, const float *theta, const float *samples,
                             double *loss, float *grad, void *hip_stream)
{
    if (n < 1 || n > (1 << 24) || !freqs || !theta || !samples) {
        set_error("irs_mlp_loss_grad: NULL argument or n outside [1, 2^24]");
        return IRS_E_INVALID;
    }
    const hipStream_t s = (hipStream_t)hip_stream;
    DevBuf<float> dth, dfr, dg;
    DevBuf<uint16_t> wf, wb;
    DevBuf<double> dl;
    TrainBufs tb;
    irs_status st;
    const int32_t bn = (int32_t)((n + 255) / 256 * 256);
    if ((st = dth.alloc(kNP)) != IRS_OK || (st = dfr.alloc(2 * kNF)) != IRS_OK ||
        (st = dg.alloc(kNP)) != IRS_OK || (st = wf.alloc((size_t)kFragFwd * 8)) != IRS_OK ||
        (st = wb.alloc((size_t)kFragBwd * 8)) != IRS_OK || (st = dl.alloc(1)) != IRS_OK ||
        (st = tb.alloc(bn)) != IRS_OK)
        return st;
    IRS_HIP(hipMemcpyAsync(dth.p, theta, sizeof(float) * kNP, hipMemcpyHostToDevice, s));
    IRS_HIP(hipMemcpyAsync(dfr.p, freqs, sizeof(float) * 2 * kNF, hipMemcpyHostToDevice, s));
    const int64_t ne = (int64_t)(kFragFwd + kFragBwd) * 8;
    hipLaunchKernelGGL(k_mlp_pack, dim3((unsigned)((ne + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       dth.p, wf.p, wb.p);
    // slots i < n take sample i (base 0, multiplier 1)
    if ((st = grad_step(s, tb, wf.p, wb.p, dth.p, dfr.p, samples, n, 0, 1, (int32_t)n, dg.p, dl.p)) != IRS_OK)
        return st;
    double l = 0.0;
    IRS_HIP(hipMemcpyAsync(&l, dl.p, sizeof(double), hipMemcpyDeviceToHost, s));
    if (grad) IRS_HIP(hipMemcpyAsync(grad, dg.p, sizeof(float) * kNP, hipMemcpyDeviceToHost, s));
    IRS_HIP(hipStreamSynchronize(s));
    if (loss) *loss = l / (double)n;
    return IRS_OK;
}

}  // extern "C"
