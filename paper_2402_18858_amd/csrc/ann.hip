// ann.hip -- the learned stand-in for DI (paper Sec. II.A "infer chemical
// source terms with ANN", Sec. II.B training data and MLP) on gfx950.
//
// Inputs per cell: the Box-Cox transform (Eq. 7, lambda = 0.1) of max(Y, 0),
// T and p, z-scored; output: the z-scored change of Y over dt.  Inference:
//   ingest (features -> BF16, envelope test, h0)   -- HBM stream, one lane/cell
//   MLP: per layer one BF16 MFMA GEMM with a fused bias+GELU epilogue
//   post (de-normalise in FP64, element projection, checks, T from h0)
//   DI on the cells routed by the envelope test or the checks.
// Training: hand-written forward (saving Z and A), MSE loss (Eq. 8) on the
// z-scored outputs, backward (dW = A^T dZ, dA = dZ W^T, GELU'), Adam on FP32
// master weights with BF16 copies for the GEMMs.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ann_internal.h"
#include "chemk.h"
#include "chemk_dev.h"
#include "chemk_internal.h"
#include "gemm.h"

using namespace chemk;

namespace {

constexpr double BCT_LAMBDA = 0.1;
constexpr int FPAD = 64;            // padded input width (GEMM K step)
constexpr int CHUNK = 65536;        // cells per MLP chunk (activations stay in the MALL)

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// x^(1/10) for x > 0 (any finite positive double, denormals included), in
// FP64 without log or exp: x = m 2^(10 q + r) with m in [0.5, 1), r in 0..9,
// so x^(1/10) = 2^q u^(1/10) with u = m 2^r in [0.5, 512).  A single-precision
// estimate of u^(1/10) from the hardware log2 and exp2 (relative error below
// 1e-6) is refined by two Newton steps on t^10 = u, t <- t (0.9 + 0.1 u / t^10)
// (quadratic: ~1e-12, then the rounding of the last step), which leaves the
// result within about 2 ulp of the exact root.
__device__ __forceinline__ double root10(double x) {
    const int e = __builtin_amdgcn_frexp_exp(x);
    const double m = __builtin_amdgcn_frexp_mant(x);
    const int q = (((e + 1100) * 6554) >> 16) - 110;   // floor(e / 10), exact for |e| < 1100
    const double u = __builtin_ldexp(m, e - 10 * q);
    double t = (double)__builtin_amdgcn_exp2f(0.1f * __builtin_amdgcn_logf((float)u));
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double t2 = t * t, t4 = t2 * t2, t10 = t4 * t4 * t2;
        double r = __builtin_amdgcn_rcp(t10);
        r = fma(r, fma(-t10, r, 1.0), r);
        t *= fma(0.1, u * r, 0.9);
    }
    return __builtin_ldexp(t, q);
}

// Box-Cox of a mass fraction (Eq. 7 with lambda = 0.1; negative round-off
// clamped to 0, NaN kept), in FP64.
static_assert(BCT_LAMBDA == 0.1, "root10 is the lambda = 0.1 power");
__device__ __forceinline__ double box_cox(double y) {
    const double r = root10(y);   // on every lane (no branch); unused for y <= 0 or NaN
    const double p = y > 0.0 ? r : (y == y ? 0.0 : y);
    return (p - 1.0) * (1.0 / BCT_LAMBDA);
}

// Element-ratio windows of the input envelope: window j holds a cell whose
// element mass fractions z_e = sum_k Emat[e][k] Y_k give
//   lo_j <= (sum_e num[j][e] z_e) / (sum_e den[j][e] z_e) <= hi_j
// with a positive denominator (molar ratios such as H/C, O/N or the elemental
// equivalence ratio: the caller folds 1/A_e into the coefficients).
constexpr int MAX_RATIOS = 4;
constexpr int RAT_E = CHEMK_MAX_ELEMENTS;
constexpr int RAT_DOUBLES = 2 * MAX_RATIOS * RAT_E + 2 * MAX_RATIOS;   // num, den, lo, hi

struct NormDev {
    const double *mu_x, *sd_x, *mu_y, *sd_y, *lo, *hi;   // [F], [F], [K], [K], [F], [F]
    const double *rat;                                   // [RAT_DOUBLES]
};

// ---------------------------------------------------------------------------
// ingest and post: one lane per cell, the cell's row in registers
// ---------------------------------------------------------------------------
// Both kernels are templated on KM >= K (16, 32 or 64: K + 2 <= FPAD bounds K
// by 62), so every loop over species is unrolled at compile time and the row
// of a cell lives in registers.  A workgroup is one wave of 64 cells; the
// rows enter and leave through LDS with coalesced global accesses.  The
// per-species constants come from a table built once per normalisation
// (zero-padded to KM), read at compile-time offsets through a restrict
// pointer: uniform scalar loads into SGPRs, which leaves the vector registers
// to the rows.
// ingest table: lo, hi, mu_x, 1/sd_x [FPAD each], nasa [7 KM], 1/W [KM],
// Emat [RAT_E KM], ratio windows [RAT_DOUBLES]
constexpr int ti_lo = 0, ti_hi = FPAD, ti_mu = 2 * FPAD, ti_sd = 3 * FPAD, ti_nasa = 4 * FPAD;
__host__ __device__ constexpr int ti_invW(int KM) { return 4 * FPAD + 7 * KM; }
__host__ __device__ constexpr int ti_elem(int KM) { return 4 * FPAD + 8 * KM; }
__host__ __device__ constexpr int ti_rat(int KM) { return 4 * FPAD + (8 + RAT_E) * KM; }
__host__ __device__ constexpr int ti_size(int KM) { return ti_rat(KM) + RAT_DOUBLES; }
constexpr int tr_num = 0, tr_den = MAX_RATIOS * RAT_E, tr_lo = 2 * MAX_RATIOS * RAT_E,
              tr_hi = 2 * MAX_RATIOS * RAT_E + MAX_RATIOS;
// post table: E [E KM], 1/W [KM], a_j (j < 6) [6 KM], mu_y [KM], sd_y [KM]
__host__ __device__ constexpr int tp_invW(int E, int KM) { return E * KM; }
__host__ __device__ constexpr int tp_a(int E, int KM) { return (E + 1) * KM; }
__host__ __device__ constexpr int tp_mu(int E, int KM) { return (E + 7) * KM; }
__host__ __device__ constexpr int tp_sd(int E, int KM) { return (E + 8) * KM; }
__host__ __device__ constexpr int tp_size(int E, int KM) { return (E + 9) * KM; }
constexpr int ROW_TAB_DOUBLES = ti_size(64) + tp_size(CHEMK_MAX_ELEMENTS, 64);

__global__ void row_tables_kernel(DevMech m, NormDev nd, int KM, double *ti, double *tp) {
    const int K = m.K, F = K + 2, E = m.E;
    for (int i = threadIdx.x; i < FPAD; i += blockDim.x) {
        const bool f = i < F;
        ti[ti_lo + i] = f ? nd.lo[i] : 0.0;
        ti[ti_hi + i] = f ? nd.hi[i] : 0.0;
        ti[ti_mu + i] = f ? nd.mu_x[i] : 0.0;
        ti[ti_sd + i] = f ? 1.0 / nd.sd_x[i] : 1.0;
    }
    for (int i = threadIdx.x; i < 7 * KM; i += blockDim.x) ti[ti_nasa + i] = i < 7 * K ? m.nasa[i] : 0.0;
    for (int i = threadIdx.x; i < RAT_DOUBLES; i += blockDim.x) ti[ti_rat(KM) + i] = nd.rat[i];
    for (int i = threadIdx.x; i < KM; i += blockDim.x) {
        const bool s = i < K;
        ti[ti_invW(KM) + i] = s ? m.invW[i] : 0.0;
        for (int e = 0; e < RAT_E; ++e) ti[ti_elem(KM) + e * KM + i] = (s && e < E) ? m.Emat[e * K + i] : 0.0;
        tp[tp_invW(E, KM) + i] = s ? m.invW[i] : 0.0;
        tp[tp_mu(E, KM) + i] = s ? nd.mu_y[i] : 0.0;
        tp[tp_sd(E, KM) + i] = s ? nd.sd_y[i] : 0.0;
        for (int j = 0; j < 6; ++j) tp[tp_a(E, KM) + j * KM + i] = s ? m.nasa[7 * i + j] : 0.0;
        for (int e = 0; e < E; ++e) tp[e * KM + i] = s ? m.Emat[e * K + i] : 0.0;
    }
}

// Features (Box-Cox of the K mass fractions, then T and p), z-scored and
// rounded to BF16 into a row of FPAD inputs; the envelope flag (a raw feature
// outside [lo, hi] of the training data, or NaN, or an element ratio outside
// its window); the enthalpy h(T, Y) / R that the post step conserves.  A
// group of KP lanes (the power of two >= K, equal to the table's KM) takes one
// cell, lane k its species k, so that the species' constants stay in the
// lane's registers for the whole launch; a wave advances 64 / KP cells per
// iteration, reading their rows of Y and writing their rows of X coalesced
// (lane k: the columns k, k + KP, ...).
constexpr int ING_THREADS = 256;

// Sum of v over the KP lanes of a group, on every lane of it: four DPP steps
// within each 16-lane row (VALU operand modifiers, no LDS round trip), then a
// swizzle across the two rows of a 32-lane half and a permute across the
// halves.  The opaque move keeps a product feeding v out of the first step.
template <int KP> __device__ __forceinline__ double group_sum(double v) {
    asm volatile("" : "+v"(v));
    v += dpp_d<kDppXor1>(v);
    v += dpp_d<kDppXor2>(v);
    v += dpp_d<kDppHalfMirror>(v);
    v += dpp_d<kDppMirror>(v);
    if (KP >= 32) {   // lanes i <-> i ^ 16 within each 32 (swizzle and_mask 31, xor_mask 16)
        const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
        const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
        v += __hiloint2double(hi, lo);
    }
    if (KP >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

template <int KP>
__global__ void __launch_bounds__(ING_THREADS) ingest_kernel(int K, int E, int nrat, int n,
                                                             const double *__restrict__ tab,
                                                             const double *__restrict__ T,
                                                             const double *__restrict__ p,
                                                             const double *__restrict__ Y,
                                                             uint16_t *__restrict__ X,
                                                             int *__restrict__ route,
                                                             double *__restrict__ h0R) {
    static_assert(KP == 16 || KP == 32 || KP == 64, "lane group");
    constexpr int CPW = 64 / KP, NCOL = FPAD / KP;
    const int lane = threadIdx.x & 63, k = lane % KP, sub = lane / KP;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int waves = gridDim.x * (ING_THREADS / 64);
    const bool sp = k < K;
    // species k's constants (zero past K) and those of the T and p features
    double lo = 0.0, hi = 0.0, mu = 0.0, isd = 0.0, iw = 0.0, a[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double em[RAT_E];
#pragma unroll
    for (int e = 0; e < RAT_E; ++e) em[e] = 0.0;
    if (sp) {
        lo = tab[ti_lo + k];
        hi = tab[ti_hi + k];
        mu = tab[ti_mu + k];
        isd = tab[ti_sd + k];
        iw = tab[ti_invW(KP) + k];
#pragma unroll
        for (int j = 0; j < 6; ++j) a[j] = tab[ti_nasa + 7 * k + j];
        if (nrat > 0) {
#pragma unroll
            for (int e = 0; e < RAT_E; ++e) em[e] = tab[ti_elem(KP) + e * KP + k];
        }
    }
    const double loT = tab[ti_lo + K], hiT = tab[ti_hi + K], muT = tab[ti_mu + K], isdT = tab[ti_sd + K];
    const double lop = tab[ti_lo + K + 1], hip = tab[ti_hi + K + 1], mup = tab[ti_mu + K + 1],
                 isdp = tab[ti_sd + K + 1];
    const unsigned long long gmask = KP == 64 ? ~0ull : ((1ull << KP) - 1ull);
    // this lane's mass fraction, T and p of group gg (the last cell past n)
    auto fetch = [&](int gg, double &y, double &Tc, double &pc) {
        const int c = gg * CPW + sub;
        const bool cv = c < n;
        const int cc = cv ? c : n - 1;
        y = (cv && sp) ? Y[(size_t)cc * K + k] : 0.0;
        Tc = T[cc];
        pc = p[cc];
    };
    int g = blockIdx.x * (ING_THREADS / 64) + wave;
    double yN = 0.0, TN = 0.0, pN = 0.0;
    if (g * CPW < n) fetch(g, yN, TN, pN);
    for (; g * CPW < n; g += waves) {
        const int c = g * CPW + sub;
        const bool cv = c < n;
        const double y = yN, Tc = TN, pc = pN;
        // the next group's loads travel during this group's arithmetic
        if ((g + waves) * CPW < n) fetch(g + waves, yN, TN, pN);
        const double raw = box_cox(y);
        double cpR, hRT;
        sp_cp_h(a, Tc, 1.0 / Tc, cpR, hRT);
        const double h = group_sum<KP>(y * iw * hRT);   // zero past K
        const bool bad = sp && !((raw >= lo) & (raw <= hi));   // NaN -> outside
        const unsigned long long m = __ballot(bad);
        bool out = ((m >> (sub * KP)) & gmask) != 0 || !((Tc >= loT) & (Tc <= hiT)) ||
                   !((pc >= lop) & (pc <= hip));
        if (nrat > 0) {   // uniform: the element-ratio windows
            double z[RAT_E];
#pragma unroll
            for (int e = 0; e < RAT_E; ++e) {
                z[e] = e < E ? group_sum<KP>(y * em[e]) : 0.0;
            }
#pragma unroll
            for (int j = 0; j < MAX_RATIOS; ++j) {
                if (j < nrat) {
                    const double *__restrict__ tr = tab + ti_rat(KP);
                    double u = 0.0, d = 0.0;
#pragma unroll
                    for (int e = 0; e < RAT_E; ++e) {
                        u += tr[tr_num + j * RAT_E + e] * z[e];
                        d += tr[tr_den + j * RAT_E + e] * z[e];
                    }
                    out = out || !((d > 0.0) & (u >= tr[tr_lo + j] * d) & (u <= tr[tr_hi + j] * d));
                }
            }
        }
        const float fs = (float)((raw - mu) * isd);
        const float fT = (float)((Tc - muT) * isdT), fp = (float)((pc - mup) * isdp);
        if (cv) {
#pragma unroll
            for (int q = 0; q < NCOL; ++q) {
                const int col = k + q * KP;   // only q = 0 can be a species column (KP >= K)
                const float v = col < K ? fs : (col == K ? fT : (col == K + 1 ? fp : 0.0f));
                X[(size_t)c * FPAD + col] = f2bf(v);
            }
            if (k == 0) {
                route[c] = out ? 1 : 0;
                h0R[c] = h * Tc;
            }
        }
    }
}

// post: the prediction y* = Y_in + dY (dY = mu + sd * out, FP64) is corrected
// to the nearest state with the input's element masses, nearness measured in
// units of each species' training spread sd_k of dY: minimise
// sum_k (y_k - y*_k)^2 / sd_k^2 subject to E y = E Y_in, whose Lagrange
// condition gives y = y* - W E^T (E W E^T)^-1 (E y* - E Y_in), W = diag(sd^2).
// Non-negativity is handled by an active set that only grows: species a solve
// leaves negative are held at zero and the correction is solved again from y*
// over the others, at most POST_SOLVES solves.  Then the admissibility checks
// (a singular solve, non-finite or Y_k < -neg_tol, a correction larger than
// adj_max sd_k on some species, T(t+dt) - T(t) outside [dT_lo, dT_hi]) and T
// from h0 by Newton; cells that fail any of it are queued for DI and left
// unchanged.
//
// One lane per cell, a wave of 64 cells per workgroup.  The rows enter and
// leave through LDS with coalesced global accesses and stay there: every pass
// over the species reads the lane's row from LDS (stride KM + 1 doubles: two
// lanes per bank at most), and the per-species constants are uniform scalar
// loads of the table, so the registers hold only the E x E system.
constexpr int POST_SOLVES = 4;
constexpr int POST_CELLS = 64;

struct PostChecks {
    double neg_tol, adj_max, dT_lo, dT_hi;
};

// Block copy of the rows of cells [0, cnt) from a row-major global span (K
// values per cell, contiguous) into an LDS tile of row stride ld, in
// consecutive global elements per lane; all of a lane's loads are issued
// before its first LDS store.  Element i is cell i / K, computed with a float
// reciprocal: exact here, since i < 4096 and the fractional part of
// (i + 0.5) / K is at least 1 / 128 away from an integer.
template <int KM, typename Tv>
__device__ __forceinline__ void rows_to_lds(const Tv *__restrict__ g, int cnt, int K, float invK,
                                            Tv *s, int ld) {
    const int total = cnt * K;
    Tv v[KM];
#pragma unroll
    for (int r = 0; r < KM; ++r) {
        const int i = r * POST_CELLS + (int)threadIdx.x;
        v[r] = i < total ? g[i] : Tv(0);
    }
#pragma unroll
    for (int r = 0; r < KM; ++r) {
        const int i = r * POST_CELLS + (int)threadIdx.x;
        if (i < total) {
            const int c = (int)(((float)i + 0.5f) * invK);
            s[c * ld + (i - c * K)] = v[r];
        }
    }
}

// Solves A x = r in place (x returned in r) by Gaussian elimination with
// partial pivoting; false if a pivot is exactly zero.
template <int E>
__device__ __forceinline__ bool solve_small(double (&A)[E][E], double (&r)[E]) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < E; ++k) {
        int piv = k;
        double best = fabs(A[k][k]);
#pragma unroll
        for (int i = k + 1; i < E; ++i)
            if (fabs(A[i][k]) > best) {
                best = fabs(A[i][k]);
                piv = i;
            }
        ok = ok && best != 0.0;
#pragma unroll
        for (int i = k + 1; i < E; ++i) {
            const bool sw = i == piv;
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const double t = A[k][j];
                A[k][j] = sw ? A[i][j] : t;
                A[i][j] = sw ? t : A[i][j];
            }
            const double t = r[k];
            r[k] = sw ? r[i] : t;
            r[i] = sw ? t : r[i];
        }
#pragma unroll
        for (int i = k + 1; i < E; ++i) {
            const double l = A[i][k] / A[k][k];
#pragma unroll
            for (int j = k; j < E; ++j) A[i][j] -= l * A[k][j];
            r[i] -= l * r[k];
        }
    }
#pragma unroll
    for (int i = E - 1; i >= 0; --i) {
#pragma unroll
        for (int j = i + 1; j < E; ++j) r[i] -= A[i][j] * r[j];
        r[i] /= A[i][i];
    }
    return ok;
}

template <int E, int KM>
__global__ void __launch_bounds__(POST_CELLS) post_kernel(int K, int n,
                                                          const double *__restrict__ tab,
                                                          double *__restrict__ T,
                                                          double *__restrict__ Y,
                                                          const float *__restrict__ out,
                                                          const int *__restrict__ route,
                                                          const double *__restrict__ h0R,
                                                          PostChecks ck, int project,
                                                          int *__restrict__ status,
                                                          int *__restrict__ nsteps,
                                                          int *__restrict__ queue,
                                                          int *__restrict__ n_routed,
                                                          unsigned long long *__restrict__ stats) {
    static_assert(KM <= 64, "held-species mask is one 64-bit word");
    constexpr int ld = KM + 1;
    __shared__ double s_y[POST_CELLS * ld];
    __shared__ float s_o[POST_CELLS * ld];
    __shared__ int s_keep[POST_CELLS];
    const int base = blockIdx.x * POST_CELLS;
    const int cnt = n - base < POST_CELLS ? n - base : POST_CELLS;
    const int lane = threadIdx.x;
    const bool valid = lane < cnt;
    const int c = valid ? base + lane : base;
    const float invK = 1.0f / (float)K;
    rows_to_lds<KM>(Y + (size_t)base * K, cnt, K, invK, s_y, ld);
    rows_to_lds<KM>(out + (size_t)base * K, cnt, K, invK, s_o, ld);
    __syncthreads();
    double *row = s_y + lane * ld;
    const float *orow = s_o + lane * ld;
    const double *__restrict__ tE = tab;
    const double *__restrict__ tmu = tab + tp_mu(E, KM);
    const double *__restrict__ tsd = tab + tp_sd(E, KM);
    // element totals of the input state (the correction's target), and the
    // row replaced by y*
    double eyin[E];
#pragma unroll
    for (int a = 0; a < E; ++a) eyin[a] = 0.0;
    for (int k = 0; k < K; ++k) {
        const double y = row[k];
#pragma unroll
        for (int a = 0; a < E; ++a) eyin[a] += tE[a * KM + k] * y;
        row[k] = y + tmu[k] + tsd[k] * (double)orow[k];
    }
    bool bad = !valid || route[c] != 0;
    // active-set solves, per lane (a lane leaves when its set stops growing);
    // lam holds the multipliers of the last solve and held its species at 0
    double lam[E];
#pragma unroll
    for (int a = 0; a < E; ++a) lam[a] = 0.0;
    unsigned long long held = 0ull;
    if (project) {
        for (int it = 0; it < POST_SOLVES; ++it) {
            double A[E][E], r[E];
#pragma unroll
            for (int a = 0; a < E; ++a) {
                r[a] = -eyin[a];
#pragma unroll
                for (int b = 0; b < E; ++b) A[a][b] = 0.0;
            }
            for (int k = 0; k < K; ++k) {
                const bool h = (held >> k) & 1ull;
                const double sd = tsd[k];
                const double w = h ? 0.0 : sd * sd;
                const double yk = h ? 0.0 : row[k];
#pragma unroll
                for (int a = 0; a < E; ++a) {
                    const double ea = tE[a * KM + k];
                    r[a] += ea * yk;
#pragma unroll
                    for (int b = 0; b <= a; ++b) A[a][b] += ea * w * tE[b * KM + k];
                }
            }
#pragma unroll
            for (int a = 0; a < E; ++a)
#pragma unroll
                for (int b = a + 1; b < E; ++b) A[a][b] = A[b][a];
            if (!solve_small<E>(A, r)) {
                bad = true;
                break;
            }
#pragma unroll
            for (int a = 0; a < E; ++a) lam[a] = r[a];
            if (it == POST_SOLVES - 1) break;
            // species this solve leaves negative
            unsigned long long neg = 0ull;
            for (int k = 0; k < K; ++k) {
                const double sd = tsd[k];
                double acc = 0.0;
#pragma unroll
                for (int a = 0; a < E; ++a) acc += tE[a * KM + k] * lam[a];
                if (!((held >> k) & 1ull) && row[k] - sd * sd * acc < 0.0) neg |= 1ull << k;
            }
            if (!neg) break;
            held |= neg;
        }
    }
    // the corrected state (back into the row), the per-species checks and the
    // mixture enthalpy polynomial: h(T) of the mixture is a NASA-7 polynomial
    // in T with coefficients B_j = sum_k (Y_k / W_k) a_jk, so each Newton
    // iteration costs one polynomial instead of one per species
    double B[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < K; ++k) {
        const double ys = row[k];
        double yk = ys;
        if (project) {
            const double sd = tsd[k];
            double acc = 0.0;
#pragma unroll
            for (int a = 0; a < E; ++a) acc += tE[a * KM + k] * lam[a];
            const bool h = (held >> k) & 1ull;
            const double corr = h ? ys : sd * sd * acc;
            yk = h ? 0.0 : ys - corr;
            if (fabs(corr) > ck.adj_max * sd) bad = true;
        }
        if (!(yk >= -ck.neg_tol) || !isfinite(yk)) bad = true;
        const double w = yk * tab[tp_invW(E, KM) + k];
#pragma unroll
        for (int j = 0; j < 6; ++j) B[j] += w * tab[tp_a(E, KM) + j * KM + k];
        row[k] = yk;
    }
    // Newton on h(T) = h0, as in the property update
    const double Tin = T[c];
    double Tn = Tin;
    if (!bad) {
        const double h0 = h0R[c];
        int st = 1;
        for (int it = 0; it < 50; ++it) {
            const double t = Tn;
            // cp/R and h/R of the mixture (per unit mass)
            const double c_ = B[0] + t * (B[1] + t * (B[2] + t * (B[3] + t * B[4])));
            const double hT = t * (B[0] + t * (B[1] * 0.5 + t * (B[2] * (1.0 / 3.0) +
                              t * (B[3] * 0.25 + t * B[4] * 0.2)))) + B[5];
            const double dT = (hT - h0) / c_;
            Tn -= dT;
            if (!isfinite(Tn)) break;
            if (fabs(dT) <= 1e-12 * fabs(Tn)) {
                if (Tn >= 200.0 && Tn <= 4000.0) st = 0;
                break;
            }
        }
        if (st || !((Tn - Tin >= ck.dT_lo) & (Tn - Tin <= ck.dT_hi))) bad = true;
    }
    // routed cells: one queue reservation per wave
    const bool rt = valid && bad;
    const unsigned long long rm = __ballot(rt);
    int slot0 = 0;
    if (lane == 0 && rm) {
        slot0 = atomicAdd(n_routed, (int)__popcll(rm));
        atomicAdd(&stats[0], (unsigned long long)__popcll(rm));
    }
    slot0 = __shfl(slot0, 0, 64);
    if (rt) {
        queue[slot0 + (int)__popcll(rm & ((1ull << lane) - 1ull))] = c;
    } else if (valid) {
        T[c] = Tn;
        status[c] = 0;
        if (nsteps) nsteps[c] = 0;
    }
    // new rows of the cells that passed; the others keep Y_in
    s_keep[lane] = (valid && !bad) ? 1 : 0;
    __syncthreads();
    double *dst = Y + (size_t)base * K;
    const int total = cnt * K;
    double v[KM];
    int kp[KM];
#pragma unroll
    for (int r = 0; r < KM; ++r) {   // all LDS reads first, then the stores
        const int i = r * POST_CELLS + lane;
        const int ii = i < total ? i : 0;
        const int cc = (int)(((float)ii + 0.5f) * invK);
        kp[r] = i < total ? s_keep[cc] : 0;
        v[r] = s_y[cc * ld + (ii - cc * K)];
    }
#pragma unroll
    for (int r = 0; r < KM; ++r)
        if (kp[r]) dst[r * POST_CELLS + lane] = v[r];
}

template <int KM> struct KmOf {
    static constexpr int v = KM;
};

// Launch helpers over the species bound KM.
static int km_of(int K) { return K <= 16 ? 16 : K <= 32 ? 32 : 64; }

template <typename Fn> static hipError_t with_km(int K, Fn &&f) {
    if (K <= 16) return f(KmOf<16>{});
    if (K <= 32) return f(KmOf<32>{});
    if (K <= 64) return f(KmOf<64>{});
    return hipErrorInvalidValue;
}

// Workgroups of ingest_kernel<KP> that are resident on the current device at
// once (CUs x workgroups per CU), found once per device and lane group.  The
// kernel's grid-stride loop then spreads the groups evenly over waves that
// all start together, instead of leaving a last round of workgroups to run
// nearly alone.
template <int KP> static int ingest_resident_grid() {
    static int cache[64] = {};   // per device; a race only writes the same value
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 2048;
    if (cache[dev] > 0) return cache[dev];
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ingest_kernel<KP>, ING_THREADS, 0) !=
            hipSuccess ||
        cus <= 0 || per_cu <= 0)
        return 2048;
    cache[dev] = cus * per_cu;
    return cache[dev];
}

static hipError_t launch_ingest(int K, int E, int nrat, const double *tab, int n, const double *T,
                                const double *p, const double *Y, uint16_t *X, int *route, double *h0,
                                hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return with_km(K, [&](auto km) {
        constexpr int KP = decltype(km)::v;
        const int64_t groups = ((int64_t)n + 64 / KP - 1) / (64 / KP);
        const int grid = (int)std::min<int64_t>(ingest_resident_grid<KP>(),
                                                (groups + ING_THREADS / 64 - 1) / (ING_THREADS / 64));
        hipLaunchKernelGGL(ingest_kernel<KP>, dim3(grid), dim3(ING_THREADS), 0, s, K, E, nrat, n, tab, T,
                           p, Y, X, route, h0);
        return hipGetLastError();
    });
}

// ---------------------------------------------------------------------------
// training helpers
// ---------------------------------------------------------------------------
__global__ void gather_rows_kernel(const int *__restrict__ idx, int B, const uint16_t *__restrict__ X,
                                   int ldx, const float *__restrict__ Z, int K, uint16_t *Xb,
                                   float *Zb) {
    const int r = blockIdx.x;
    if (r >= B) return;
    const int src = idx[r];
    for (int k = threadIdx.x; k < ldx; k += blockDim.x) Xb[(size_t)r * ldx + k] = X[(size_t)src * ldx + k];
    for (int k = threadIdx.x; k < K; k += blockDim.x) Zb[(size_t)r * K + k] = Z[(size_t)src * K + k];
}

// Where a batch's loss goes: loss_acc[0], or with ctl the slot of the current
// epoch, loss_acc[ctl[0] / spe], scaled by `scale` (1 / batches per epoch).
struct LossSink {
    float *acc;
    const long long *ctl;
    int spe;
    float scale;
};

// MSE on z-scored outputs: loss = mean((out - tgt)^2); dOut = bf16(2 (out - tgt) / count)
// gscale = 1: the gradient of the mean over all count values; gscale = G for
// G networks side by side, each with the mean over its own count / G values
// (the loss reported stays the mean over all).
__global__ void mse_kernel(const float *__restrict__ out, const float *__restrict__ tgt, int count,
                           uint16_t *dout, LossSink sink, float gscale = 1.0f) {
    __shared__ float red[256];
    float s = 0.f;
    const float sc = 2.0f * gscale / (float)count;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const float d = out[i] - tgt[i];
        s += d * d;
        dout[i] = f2bf(d * sc);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && sink.acc) {
        float *dst = sink.ctl ? sink.acc + sink.ctl[0] / sink.spe : sink.acc;
        atomicAdd(dst, red[0] / (float)count * sink.scale);
    }
}

// The loss of Eq. 11 with the physics terms (chemk_ann_train_step): one thread
// per row.  d = out - tgt; data term mean(d^2) over the B K values; mass term
// w_mass |m| / S with m = sum_k (mu_k + sd_k out_k) and S = sum_k sd_k; heat
// release term w_hrr e^2 with e = sum_k G_k d_k; both averaged over rows.
// dOut = bf16 of the gradient of the total, rounded once.
__global__ void phys_loss_kernel(const float *__restrict__ out, const float *__restrict__ tgt,
                                 const float *__restrict__ G, const float *__restrict__ ow, float inv_wsum, int B,
                                 int K, const double *__restrict__ mu, const double *__restrict__ sd, float inv_S,
                                 float w_mass, float w_hrr, uint16_t *dout, LossSink sink) {
    __shared__ float red[256];
    float s = 0.f;
    // data term: sum_k w_k d_k^2 / (B sum_k w_k), w_k = 1 without per-output weights
    const float sc = 2.0f * inv_wsum / (float)B, rb = 1.0f / (float)B;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B; i += gridDim.x * blockDim.x) {
        const float *o = out + (size_t)i * K, *t = tgt + (size_t)i * K;
        const float *g = G ? G + (size_t)i * K : nullptr;
        float dd = 0.f, m = 0.f, e = 0.f;
        for (int k = 0; k < K; ++k) {
            const float d = o[k] - t[k];
            dd += (ow ? ow[k] : 1.f) * d * d;
            m += (float)mu[k] + (float)sd[k] * o[k];
            if (g) e += g[k] * d;
        }
        s += dd * inv_wsum * rb + w_mass * fabsf(m) * inv_S * rb + (g ? w_hrr * e * e * rb : 0.f);
        const float cm = w_mass * (m > 0.f ? 1.f : (m < 0.f ? -1.f : 0.f)) * inv_S * rb;
        const float ce = g ? 2.0f * w_hrr * e * rb : 0.f;
        for (int k = 0; k < K; ++k) {
            const float gr = (ow ? ow[k] : 1.f) * (o[k] - t[k]) * sc + cm * (float)sd[k] + (g ? ce * g[k] : 0.f);
            dout[(size_t)i * K + k] = f2bf(gr);
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o2 = blockDim.x / 2; o2 > 0; o2 >>= 1) {
        if ((int)threadIdx.x < o2) red[threadIdx.x] += red[threadIdx.x + o2];
        __syncthreads();
    }
    if (threadIdx.x == 0 && sink.acc) {
        float *dst = sink.ctl ? sink.acc + sink.ctl[0] / sink.spe : sink.acc;
        atomicAdd(dst, red[0] * sink.scale);
    }
}

// Rows idx[0..B-1] of G [., K] into Gb [B, K].
__global__ void gather_g_kernel(const int *__restrict__ idx, int B, const float *__restrict__ G, int K,
                                float *Gb) {
    const int r = blockIdx.x;
    if (r >= B) return;
    const int src = idx[r];
    for (int k = threadIdx.x; k < K; k += blockDim.x) Gb[(size_t)r * K + k] = G[(size_t)src * K + k];
}

// Heat release over the step of row i (chemk_ann_hrr_weights): the label
// HRR_i = -(rho/dt) sum_k h_k dY_k, its square added to *sum2; with scale > 0
// also the row of weights G_ik = -(rho/dt) h_k sd_k / scale.  One thread per row.
__global__ void hrr_weights_kernel(DevMech m, int n, const double *__restrict__ T, const double *__restrict__ p,
                                   const double *__restrict__ Y, const double *__restrict__ Yn, double dt,
                                   const double *__restrict__ sd, double scale, float *G, double *sum2) {
    const int K = m.K;
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double Ti = T[i], invT = 1.0 / Ti;
        double ws = 0.0, q = 0.0;
        for (int k = 0; k < K; ++k) ws += Y[(size_t)i * K + k] * m.invW[k];
        // rho [kg/m^3] = p Wbar / (R T) with Wbar in kg/mol
        const double rdt = p[i] * 1e-3 / (ws * RU_SI * Ti) / dt;
        for (int k = 0; k < K; ++k) {
            double cpR, hRT;
            sp_cp_h(m.nasa + 7 * k, Ti, invT, cpR, hRT);
            const double hk = hRT * RU_SI * Ti * 1e3 * m.invW[k];   // J/kg
            if (Yn) q -= rdt * hk * (Yn[(size_t)i * K + k] - Y[(size_t)i * K + k]);
            if (scale > 0.0) G[(size_t)i * K + k] = (float)(-rdt * hk * sd[k] / scale);
        }
        acc += q * q;
    }
    if (sum2) atomicAdd(sum2, acc);
}

// Sum over `count` values of (out - tgt)^2 / denom into *acc (held-out loss).
__global__ void sq_err_kernel(const float *__restrict__ out, const float *__restrict__ tgt,
                              long long count, double denom, float *acc) {
    __shared__ float red[256];
    float s = 0.f;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x) {
        const float d = out[i] - tgt[i];
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(acc, (float)(red[0] / denom));
}

__global__ void zero_f32_kernel(float *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// ---------------------------------------------------------------------------
// the training loop's device-side schedule
// ---------------------------------------------------------------------------
// ctl[0] = steps done in this training call, ctl[1] = optimizer steps before
// it.  Every step's kernels read them, so one captured step is replayed for
// all steps.

// SplitMix64's output function (Steele, Lea, Flood 2014): a bijective 64-bit
// mixer, the round function of the permutation below.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// A pseudo-random permutation of [0, n): a four-round balanced Feistel
// network on 2 * half bits (2^(2 half) >= n) keyed by `key`, with cycle
// walking (values >= n are mapped again until they fall inside; the walk ends
// because the cycle through i comes back to i < n).
__device__ __forceinline__ unsigned int feistel_perm(unsigned int i, unsigned int n, int half,
                                                     unsigned long long key) {
    const unsigned int mask = (1u << half) - 1u;
    unsigned int x = i;
    do {
        unsigned int L = x >> half, R = x & mask;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const unsigned int t =
                L ^ (unsigned int)(mix64(key + 0x9e3779b97f4a7c15ull * (unsigned long long)(r + 1) + R) & mask);
            L = R;
            R = t;
        }
        x = (L << half) | R;
    } while (x >= n);
    return x;
}

// Rows of the current step's batch: epoch e = s / spe, batch b = s % spe,
// row r -> perm_e(b B + r) with the epoch's key mix64(seed ^ mix64(e + 1)).
__global__ void batch_index_kernel(const long long *ctl, int B, int spe, unsigned int n, int half,
                                   unsigned long long seed, int *idx) {
    const long long st = ctl[0];
    const unsigned long long e = (unsigned long long)(st / spe);
    const unsigned int b = (unsigned int)(st % spe);
    const unsigned long long key = mix64(seed ^ mix64(e + 1ull));
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < B; r += gridDim.x * blockDim.x)
        idx[r] = (int)feistel_perm(b * (unsigned int)B + (unsigned int)r, n, half, key);
}

// Adam (Kingma & Ba 2015, Alg. 1) with the step count t = ctl[1] + ctl[0] + 1
// and the cosine learning rate lr1 + (lr0 - lr1)(1 + cos(pi s / total)) / 2,
// s = ctl[0], both read from the device.
// The BF16 operand copies of one network's layers, refreshed by the Adam
// pass that updates their masters (adam_sched_kernel): a weight at master
// index woff[l] + r out[l] + c goes to Wb[l][r out[l] + c] and
// Wt[l][c in[l] + r].  L = 0: no copies (refreshed apart).
struct CastTable {
    int L;
    long long woff[16], boff[16];
    int in[16], out[16];
    uint16_t *Wt[16], *Wb[16];
};

__global__ void adam_sched_kernel(float *p, const float *__restrict__ g, float *mo, float *vo, int64_t n,
                                  const long long *ctl, double lr0, double lr1, long long total, double b1d,
                                  double b2d, float eps, CastTable ct) {
    __shared__ float sh[3];
    const float b1 = (float)b1d, b2 = (float)b2d;
    if (threadIdx.x == 0) {
        const long long st = ctl[0];
        const double t = (double)(ctl[1] + st + 1);
        const double lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + cos(M_PI * (double)st / (double)(total > 0 ? total : 1)));
        sh[0] = (float)lr;
        sh[1] = (float)(1.0 / (1.0 - pow(b1d, t)));
        sh[2] = (float)(1.0 / (1.0 - pow(b2d, t)));
    }
    __syncthreads();
    const float lr = sh[0], bc1 = sh[1], bc2 = sh[2];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float m = b1 * mo[i] + (1.f - b1) * gi;
        const float v = b2 * vo[i] + (1.f - b2) * gi * gi;
        mo[i] = m;
        vo[i] = v;
        const float pn = p[i] - lr * (m * bc1) / (sqrtf(v * bc2) + eps);
        p[i] = pn;
        for (int l = 0; l < ct.L; ++l)
            if (i >= ct.woff[l] && i < ct.boff[l]) {
                const int e = (int)(i - ct.woff[l]);
                const int r = e / ct.out[l], c = e - r * ct.out[l];
                const uint16_t b = f2bf(pn);
                ct.Wb[l][e] = b;
                ct.Wt[l][(size_t)c * ct.in[l] + r] = b;
                break;
            }
    }
}

__global__ void step_end_kernel(long long *ctl) {
    if (threadIdx.x == 0) ctl[0] += 1;
}

// ctl[0]: the step within the schedule (starting at step0); ctl[1] + ctl[0]
// + 1: Adam's step count (before: the context's steps so far)
__global__ void ctl_init_kernel(long long *ctl, long long step0, long long before) {
    if (threadIdx.x == 0) {
        ctl[0] = step0;
        ctl[1] = before - step0;
    }
}

// db[o] = sum_b dZ[b][o] (FP32 accumulation of the BF16 gradient) in two
// passes with a fixed order: block row y sums rows [y R, (y + 1) R) of a
// 256-column slab into part[y][o] (a row of 256 columns per load, coalesced),
// then part is summed over y in order.
constexpr int COLSUM_ROWS = 64;

__global__ void colsum_part_kernel(const uint16_t *__restrict__ dZ, int B, int N, float *part) {
    const int b0 = blockIdx.y * COLSUM_ROWS;
    const int rows = B - b0 < COLSUM_ROWS ? B - b0 : COLSUM_ROWS;
    if (N % 8 == 0) {
        // eight columns per thread, one 16-byte load per row; rows summed in order
        const int o = 8 * (blockIdx.x * blockDim.x + threadIdx.x);
        if (o >= N) return;
        float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        const uint16_t *p = dZ + (size_t)b0 * N + o;
#pragma unroll 8
        for (int i = 0; i < rows; ++i) {
            const uint4 v = *reinterpret_cast<const uint4 *>(p + (size_t)i * N);
            s[0] += __uint_as_float(v.x << 16);
            s[1] += __uint_as_float(v.x & 0xffff0000u);
            s[2] += __uint_as_float(v.y << 16);
            s[3] += __uint_as_float(v.y & 0xffff0000u);
            s[4] += __uint_as_float(v.z << 16);
            s[5] += __uint_as_float(v.z & 0xffff0000u);
            s[6] += __uint_as_float(v.w << 16);
            s[7] += __uint_as_float(v.w & 0xffff0000u);
        }
        float *q = part + (size_t)blockIdx.y * N + o;
#pragma unroll
        for (int j = 0; j < 8; ++j) q[j] = s[j];
        return;
    }
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= N) return;
    float s = 0.f;
    for (int i = 0; i < rows; ++i) s += bf2f(dZ[(size_t)(b0 + i) * N + o]);
    part[(size_t)blockIdx.y * N + o] = s;
}

// db[(o / w) gstride + o % w] = sum over the row partials of column o: w = N
// for one network, w = the width of one of the networks side by side
__global__ void colsum_final_kernel(const float *__restrict__ part, int P, int N, float *db, int w = 0,
                                    size_t gstride = 0) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= N) return;
    float s = 0.f;
#pragma unroll 16
    for (int y = 0; y < P; ++y) s += part[(size_t)y * N + o];
    if (w > 0) db[(size_t)(o / w) * gstride + o % w] = s;
    else db[o] = s;
}

// dst[c ldd + r] = src[r lds + c] for r < R, c < C (BF16), through a 64 x 64
// LDS tile: both the reads and the writes go along rows
constexpr int TP_TILE = 64;
__global__ void __launch_bounds__(256) transpose_bf16_kernel(const uint16_t *__restrict__ src, int R, int C,
                                                             int lds, uint16_t *__restrict__ dst, int ldd) {
    __shared__ uint16_t t[TP_TILE][TP_TILE + 2];
    const int c0 = blockIdx.x * TP_TILE, r0 = blockIdx.y * TP_TILE;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
    for (int i = ty; i < TP_TILE; i += 4) {
        const int r = r0 + i, c = c0 + tx;
        t[i][tx] = (r < R && c < C) ? src[(size_t)r * lds + c] : (uint16_t)0;
    }
    __syncthreads();
#pragma unroll
    for (int i = ty; i < TP_TILE; i += 4) {
        const int c = c0 + i, r = r0 + tx;
        if (c < C && r < R) dst[(size_t)c * ldd + r] = t[tx][i];
    }
}

// grad[g gstride + r] = D[(g n + r) G + g], r < n: the diagonal blocks of the
// dense output-layer weight gradient of G networks side by side
__global__ void diag_blocks_kernel(const float *__restrict__ D, int n, int G, float *grad, size_t gstride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * G) return;
    const int g = i / n, r = i - g * n;
    grad[(size_t)g * gstride + r] = D[((size_t)g * n + r) * G + g];
}

// Adam (Kingma & Ba 2015, Alg. 1) on the FP32 master parameters.
__global__ void adam_kernel(float *p, const float *__restrict__ g, float *mo, float *vo, int64_t n,
                            float lr, float b1, float b2, float eps, float bc1, float bc2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float m = b1 * mo[i] + (1.f - b1) * gi;
        const float v = b2 * vo[i] + (1.f - b2) * gi * gi;
        mo[i] = m;
        vo[i] = v;
        p[i] -= lr * (m * bc1) / (sqrtf(v * bc2) + eps);
    }
}

// BF16 copies of one layer: Wt [out x in] (forward, K-contiguous) and W [in x out]
// dst[g n + j] = src[g stride + j] rounded to BF16 (kept as FP32), j < n, g < G
__global__ void bf16_rows_kernel(const float *__restrict__ src, size_t stride, int n, int G, float *dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * G) return;
    const int g = i / n, j = i - g * n;
    dst[i] = __uint_as_float((uint32_t)f2bf(src[g * stride + j]) << 16);
}

// out[r, g] = sum_p P[r, g S + p] (p ascending) + b[g]: the per-species
// networks' outputs from the fused last hidden layer's partial sums
__global__ void species_out_kernel(const float *__restrict__ P, int S, int G, int rows,
                                   const float *__restrict__ b, float *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * G) return;
    const int g = i % G;
    const float *p = P + (size_t)i * S;
    float s = 0.f;
    for (int k = 0; k < S; ++k) s += p[k];
    out[i] = s + b[g];
}

// Network g = blockIdx.y of an ensemble, element i = r out + c of its layer
// block [in x out] in the master: v = bf16(W); Wt[g wtG + c in + r] = v and,
// when Wb is given, Wb[g wbG + r wbLd + c] = v.
__global__ void cast_group_kernel(const float *__restrict__ M, size_t gstride, int in, int out, uint16_t *Wt,
                                  size_t wtG, uint16_t *Wb, size_t wbG, int wbLd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= in * out) return;
    const size_t g = blockIdx.y;
    const int r = i / out, c = i - r * out;
    const uint16_t v = f2bf(M[g * gstride + i]);
    Wt[g * wtG + (size_t)c * in + r] = v;
    if (Wb) Wb[g * wbG + (size_t)r * wbLd + c] = v;
}

// The same for a layer with out > 1, through a 64 x 64 LDS tile per block so
// that the transposed Wt writes go along rows: block (bx, by, g) takes rows
// [64 by, +64) and columns [64 bx, +64) of network g's [in x out] block.
__global__ void __launch_bounds__(256) cast_group_tiled_kernel(const float *__restrict__ M, size_t gstride, int in,
                                                               int out, uint16_t *Wt, size_t wtG, uint16_t *Wb,
                                                               size_t wbG, int wbLd) {
    __shared__ uint16_t t[64][66];
    const size_t g = blockIdx.z;
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const float *Mg = M + g * gstride;
#pragma unroll
    for (int i = ty; i < 64; i += 4) {
        const int r = r0 + i, c = c0 + tx;
        uint16_t v = 0;
        if (r < in && c < out) {
            v = f2bf(Mg[(size_t)r * out + c]);
            if (Wb) Wb[g * wbG + (size_t)r * wbLd + c] = v;
        }
        t[i][tx] = v;
    }
    __syncthreads();
#pragma unroll
    for (int i = ty; i < 64; i += 4) {
        const int c = c0 + i, r = r0 + tx;
        if (c < out && r < in) Wt[g * wtG + (size_t)c * in + r] = t[tx][i];
    }
}

__global__ void cast_layer_kernel(const float *__restrict__ Wm, int in, int out, uint16_t *Wt,
                                  uint16_t *Wb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= in * out) return;
    const int r = i / out, c = i - r * out;
    const uint16_t v = f2bf(Wm[i]);
    if (Wb) Wb[i] = v;
    Wt[(size_t)c * in + r] = v;
}

// ---------------------------------------------------------------------------
// normalisation statistics and envelope
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long ordered(double v) {
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double unordered(unsigned long long u) {
    u = (u & 0x8000000000000000ull) ? (u & 0x7fffffffffffffffull) : ~u;
    return __longlong_as_double((long long)u);
}

// feature j of pair c: raw inputs (j < F) then dY (j >= F)
__device__ __forceinline__ double pair_feature(int K, int j, int c, const double *T, const double *p,
                                               const double *Y, const double *Yn) {
    const int F = K + 2;
    if (j < K) return box_cox(Y[(size_t)c * K + j]);
    if (j == K) return T[c];
    if (j == K + 1) return p[c];
    const int k = j - F;
    return Yn[(size_t)c * K + k] - Y[(size_t)c * K + k];
}

// pass 0: sums (and min/max); pass 1: sums of squared deviations
__global__ void stats_kernel(int K, int n, const double *T, const double *p, const double *Y,
                             const double *Yn, int pass, const double *mean, double *acc,
                             unsigned long long *mn, unsigned long long *mx) {
    const int nf = 2 * K + 2;
    const int j = blockIdx.y;
    if (j >= nf) return;
    __shared__ double red[256];
    __shared__ unsigned long long rmn[256], rmx[256];
    double s = 0.0;
    unsigned long long lmn = ~0ull, lmx = 0ull;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        const double v = pair_feature(K, j, c, T, p, Y, Yn);
        if (pass == 0) {
            s += v;
            const unsigned long long o = ordered(v);
            lmn = o < lmn ? o : lmn;
            lmx = o > lmx ? o : lmx;
        } else {
            const double d = v - mean[j];
            s += d * d;
        }
    }
    red[threadIdx.x] = s;
    rmn[threadIdx.x] = lmn;
    rmx[threadIdx.x] = lmx;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[threadIdx.x] += red[threadIdx.x + o];
            rmn[threadIdx.x] = rmn[threadIdx.x + o] < rmn[threadIdx.x] ? rmn[threadIdx.x + o] : rmn[threadIdx.x];
            rmx[threadIdx.x] = rmx[threadIdx.x + o] > rmx[threadIdx.x] ? rmx[threadIdx.x + o] : rmx[threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&acc[j], red[0]);
        if (pass == 0) {
            atomicMin(&mn[j], rmn[0]);
            atomicMax(&mx[j], rmx[0]);
        }
    }
}

__global__ void stats_finish_kernel(int nf, int n, double *acc, double *mean, int pass) {
    const int j = threadIdx.x + blockIdx.x * blockDim.x;
    if (j >= nf) return;
    if (pass == 0) mean[j] = acc[j] / n;
    else mean[j] = sqrt(acc[j] / n);
}

__global__ void decode_minmax_kernel(int nf, const unsigned long long *mn, const unsigned long long *mx,
                                     double *lo, double *hi) {
    const int j = threadIdx.x + blockIdx.x * blockDim.x;
    if (j >= nf) return;
    lo[j] = unordered(mn[j]);
    hi[j] = unordered(mx[j]);
}

// Values whose quantiles make the envelope: raw feature j < F of state c,
// then the element-ratio windows (valid where the denominator is positive),
// then T_next - T.
struct EnvSrc {
    int K, E, F, nrat, has_dT, n;
    const double *T, *p, *Y, *Tn, *Emat;   // Emat [E*K]
    double num[MAX_RATIOS * RAT_E], den[MAX_RATIOS * RAT_E];
};

__device__ __forceinline__ bool env_value(const EnvSrc &s, int j, int c, double &v) {
    if (j < s.K) {
        v = box_cox(s.Y[(size_t)c * s.K + j]);
        return true;
    }
    if (j == s.K) {
        v = s.T[c];
        return true;
    }
    if (j == s.K + 1) {
        v = s.p[c];
        return true;
    }
    const int r = j - s.F;
    if (r < s.nrat) {
        double u = 0.0, d = 0.0;
        for (int e = 0; e < s.E; ++e) {
            double z = 0.0;
            for (int k = 0; k < s.K; ++k) z += s.Emat[e * s.K + k] * s.Y[(size_t)c * s.K + k];
            u += s.num[r * RAT_E + e] * z;
            d += s.den[r * RAT_E + e] * z;
        }
        v = u / d;
        return d > 0.0 && isfinite(v);
    }
    v = s.Tn[c] - s.T[c];
    return isfinite(v);
}

// pass 0: minimum, maximum (order-preserving integer keys) and count of the
// valid values of value j = blockIdx.y
__global__ void env_range_kernel(EnvSrc s, unsigned long long *mn, unsigned long long *mx,
                                 unsigned long long *cnt) {
    const int j = blockIdx.y;
    __shared__ unsigned long long rmn[256], rmx[256], rc[256];
    unsigned long long lmn = ~0ull, lmx = 0ull, lc = 0ull;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < s.n; c += gridDim.x * blockDim.x) {
        double v;
        if (env_value(s, j, c, v)) {
            const unsigned long long o = ordered(v);
            lmn = o < lmn ? o : lmn;
            lmx = o > lmx ? o : lmx;
            lc += 1;
        }
    }
    rmn[threadIdx.x] = lmn;
    rmx[threadIdx.x] = lmx;
    rc[threadIdx.x] = lc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            rmn[threadIdx.x] = rmn[threadIdx.x + o] < rmn[threadIdx.x] ? rmn[threadIdx.x + o] : rmn[threadIdx.x];
            rmx[threadIdx.x] = rmx[threadIdx.x + o] > rmx[threadIdx.x] ? rmx[threadIdx.x + o] : rmx[threadIdx.x];
            rc[threadIdx.x] += rc[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMin(&mn[j], rmn[0]);
        atomicMax(&mx[j], rmx[0]);
        atomicAdd(&cnt[j], rc[0]);
    }
}

constexpr int ENV_BINS = 4096;

__device__ __forceinline__ int env_bin(double v, double lo, double hi) {
    const double t = hi > lo ? (v - lo) / (hi - lo) * ENV_BINS : 0.0;
    int b = (int)t;
    return b < 0 ? 0 : (b >= ENV_BINS ? ENV_BINS - 1 : b);
}

// pass 1: histogram of value j over ENV_BINS equal bins between its
// minimum and maximum (per block in LDS, then added to the global one)
__global__ void env_hist_kernel(EnvSrc s, const unsigned long long *mn, const unsigned long long *mx,
                                unsigned int *hist) {
    const int j = blockIdx.y;
    __shared__ unsigned int h[ENV_BINS];
    for (int i = threadIdx.x; i < ENV_BINS; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    const double lo = unordered(mn[j]), hi = unordered(mx[j]);
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < s.n; c += gridDim.x * blockDim.x) {
        double v;
        if (env_value(s, j, c, v)) atomicAdd(&h[env_bin(v, lo, hi)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ENV_BINS; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[(size_t)j * ENV_BINS + i], h[i]);
}

// pass 2 (one thread per value): the bins holding the ranks floor(q cnt) from
// either end; lo = lower edge of the first, hi = upper edge of the second
__global__ void env_quantile_kernel(int nv, const unsigned long long *mn, const unsigned long long *mx,
                                    const unsigned long long *cnt, const unsigned int *hist, double q,
                                    double *qlo, double *qhi) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    const double lo = unordered(mn[j]), hi = unordered(mx[j]);
    if (cnt[j] == 0) {
        qlo[j] = NAN;
        qhi[j] = NAN;
        return;
    }
    const unsigned long long skip = (unsigned long long)(q * (double)cnt[j]);
    const unsigned int *h = hist + (size_t)j * ENV_BINS;
    const double w = (hi - lo) / ENV_BINS;
    unsigned long long acc = 0ull;
    int blo = 0, bhi = ENV_BINS - 1;
    for (int b = 0; b < ENV_BINS; ++b) {
        acc += h[b];
        if (acc > skip) {
            blo = b;
            break;
        }
    }
    acc = 0ull;
    for (int b = ENV_BINS - 1; b >= 0; --b) {
        acc += h[b];
        if (acc > skip) {
            bhi = b;
            break;
        }
    }
    qlo[j] = blo == 0 ? lo : lo + w * blo;
    qhi[j] = bhi == ENV_BINS - 1 ? hi : lo + w * (bhi + 1);
}

// training targets: z-scored dY, FP32
__global__ void pack_targets_kernel(int K, int n, const double *Y, const double *Yn,
                                    const double *mu_y, const double *sd_y, float *Z) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)n * K;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(i % K);
        Z[i] = (float)((Yn[i] - Y[i] - mu_y[k]) / sd_y[k]);
    }
}

// the step's counters in one launch: routed count, DI queue counter, stats[4]
__global__ void reset_step_kernel(int *n_routed, int *counter, unsigned long long *stats) {
    const int t = threadIdx.x;
    if (t == 0) *n_routed = 0;
    if (t == 1) *counter = 0;
    if (t < 4) stats[t] = 0ull;
}

}  // namespace

// ---------------------------------------------------------------------------
// state
// ---------------------------------------------------------------------------
struct AnnState {
    int K = 0, F = 0, L = 0;
    // G = 1: one network with K outputs.  G = K: one network per species
    // (dims[L] = 1), run together for inference only; master then holds G
    // copies of the one-network layout, gstride floats apart.
    int G = 1;
    size_t gstride = 0;
    std::vector<float *> eB;          // ensemble biases per layer [G pd[l+1]]
    float *eW = nullptr;              // output weights, BF16-rounded, [G pd[L-1]] (L >= 3)
    float *eP = nullptr;              // partial output sums of the fused last hidden layer
    std::vector<int> dims;       // logical, dims[0] = K + 2
    std::vector<int> pd;         // internal: pd[0] = FPAD
    std::vector<size_t> woff, boff;   // offsets (floats) of W_l, b_l in the master vector
    size_t nparam = 0, npublic = 0;
    float *master = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
    std::vector<uint16_t *> Wt, Wb;   // BF16 copies per layer
    // normalisation and envelope (device: mu_x, sd_x, mu_y, sd_y, lo, hi)
    double *normdev = nullptr;
    double *rowtab = nullptr;    // per-species tables of the ingest and post kernels
    bool rowtab_stale = true;
    std::vector<double> mu_x, sd_x, mu_y, sd_y, lo, hi;
    double dt = 0.0, neg_tol = 1e-6;
    chemk_ann_checks checks{};   // output checks and element-ratio windows
    // Changes whenever something a captured step graph holds by value or by
    // address changes (buffers, tables, checks): part of the graph cache key.
    uint64_t generation = 1;
    bool have_w = false, have_norm = false, have_env = false;
    long step = 0;
    // inference scratch
    int64_t cap = 0;
    uint16_t *X = nullptr;
    int *route = nullptr;
    double *h0 = nullptr;
    float *out = nullptr;
    uint16_t *act[2] = {nullptr, nullptr};
    // training scratch
    int tB = 0;
    uint16_t *tX = nullptr;
    std::vector<uint16_t *> tdZ;      // dLoss/dZ of each layer's output [B x pd[l+1]]
    float *tZt = nullptr, *tOut = nullptr, *tLoss = nullptr, *tGt = nullptr;
    float *tWork = nullptr;           // per layer: split-K partials, then column-sum partials
    std::vector<size_t> tWoff;        // offset of layer l's region in tWork
    // in a captured step the weight gradients run beside the chain of input
    // gradients: layer l's on side stream l % 4, forked after its dZ and
    // joined before Adam
    hipStream_t side[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<hipEvent_t> evFork, evJoin;
    // per-species networks: transposed activations and dZ of the layer whose
    // weight gradient is being formed ([width x B], batch contiguous)
    uint16_t *tT[2] = {nullptr, nullptr};
    std::vector<float *> tZ;          // pre-activations per hidden layer
    std::vector<uint16_t *> tA;       // activations per layer input
};

static thread_local std::string g_ann_err;

static int afail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_ann_err = buf;
    return code;
}

const char *ann_last_error() { return g_ann_err.c_str(); }

void ann_destroy(AnnState *a) {
    if (!a) return;
    (void)hipFree(a->master);
    (void)hipFree(a->grad);
    (void)hipFree(a->m1);
    (void)hipFree(a->m2);
    for (auto p : a->Wt) (void)hipFree(p);
    for (auto p : a->Wb) (void)hipFree(p);
    for (auto p : a->eB) (void)hipFree(p);
    (void)hipFree(a->eW);
    (void)hipFree(a->eP);
    (void)hipFree(a->normdev);
    (void)hipFree(a->rowtab);
    (void)hipFree(a->X);
    (void)hipFree(a->route);
    (void)hipFree(a->h0);
    (void)hipFree(a->out);
    (void)hipFree(a->act[0]);
    (void)hipFree(a->act[1]);
    (void)hipFree(a->tX);
    for (auto p : a->tdZ) (void)hipFree(p);
    (void)hipFree(a->tZt);
    (void)hipFree(a->tGt);
    (void)hipFree(a->tOut);
    (void)hipFree(a->tLoss);
    (void)hipFree(a->tWork);
    for (auto p : a->tZ) (void)hipFree(p);
    for (size_t i = 1; i < a->tA.size(); ++i) (void)hipFree(a->tA[i]);   // tA[0] aliases tX
    (void)hipFree(a->tT[0]);
    (void)hipFree(a->tT[1]);
    for (auto st : a->side)
        if (st) (void)hipStreamDestroy(st);
    for (auto ev : a->evFork) (void)hipEventDestroy(ev);
    for (auto ev : a->evJoin) (void)hipEventDestroy(ev);
    delete a;
}

bool ann_ready(const AnnState *a) { return a && a->have_w && a->have_norm; }
double ann_dt(const AnnState *a) { return a ? a->dt : 0.0; }

// BF16 product operands and gathered biases of the G networks of an ensemble
static hipError_t refresh_ensemble(AnnState *a, hipStream_t s) {
    const int G = a->G, L = a->L;
    for (int l = 0; l < L; ++l) {
        const int in = a->pd[l], out = a->pd[l + 1];
        const bool last = l == L - 1;   // out = 1: block-diagonal placement
        const size_t wtG = last ? (size_t)(G + 1) * in : (size_t)in * out;
        const size_t wbG = last ? (size_t)in * G + 1 : (size_t)in * out;
        if (last)   // out = 1: Wt runs along r already
            hipLaunchKernelGGL(cast_group_kernel, dim3((in * out + 255) / 256, G), dim3(256), 0, s,
                               a->master + a->woff[l], a->gstride, in, out, a->Wt[l], wtG, a->Wb[l], wbG, G);
        else
            hipLaunchKernelGGL(cast_group_tiled_kernel, dim3((out + 63) / 64, (in + 63) / 64, G), dim3(256), 0, s,
                               a->master + a->woff[l], a->gstride, in, out, a->Wt[l], wtG, a->Wb[l], wbG, out);
        hipError_t e = hipMemcpy2DAsync(a->eB[l], 4 * (size_t)out, a->master + a->boff[l], 4 * a->gstride,
                                        4 * (size_t)out, G, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    if (a->eW) {
        const int n = a->pd[L - 1];
        hipLaunchKernelGGL(bf16_rows_kernel, dim3((n * G + 255) / 256), dim3(256), 0, s,
                           a->master + a->woff[L - 1], a->gstride, n, G, a->eW);
    }
    return hipGetLastError();
}

// partial sums per row and network of the fused last hidden layer: two per
// 128-column tile of its padded width
static int species_slots(const AnnState *a) { return 2 * ((a->pd[a->L - 1] + 127) / 128); }

static hipError_t refresh_bf16(AnnState *a, hipStream_t s) {
    if (a->G > 1) return refresh_ensemble(a, s);
    for (int l = 0; l < a->L; ++l) {
        const int in = a->pd[l], out = a->pd[l + 1];
        hipLaunchKernelGGL(cast_layer_kernel, dim3((in * out + 255) / 256), dim3(256), 0, s,
                           a->master + a->woff[l], in, out, a->Wt[l], a->Wb[l]);
    }
    return hipGetLastError();
}

static uint64_t next_generation() {
    static std::atomic<uint64_t> g{1};
    return ++g;
}

static size_t normdev_doubles(const AnnState *a) { return 4 * a->F + 2 * a->K + RAT_DOUBLES; }

static NormDev norm_dev(const AnnState *a) {
    const int F = a->F, K = a->K;
    NormDev nd;
    nd.mu_x = a->normdev;
    nd.sd_x = a->normdev + F;
    nd.mu_y = a->normdev + 2 * F;
    nd.sd_y = a->normdev + 2 * F + K;
    nd.lo = a->normdev + 2 * F + 2 * K;
    nd.hi = a->normdev + 3 * F + 2 * K;
    nd.rat = a->normdev + 4 * F + 2 * K;
    return nd;
}

static hipError_t upload_norm(AnnState *a) {
    const int F = a->F, K = a->K;
    std::vector<double> h(normdev_doubles(a), 0.0);
    std::memcpy(h.data(), a->mu_x.data(), 8 * F);
    std::memcpy(h.data() + F, a->sd_x.data(), 8 * F);
    std::memcpy(h.data() + 2 * F, a->mu_y.data(), 8 * K);
    std::memcpy(h.data() + 2 * F + K, a->sd_y.data(), 8 * K);
    std::memcpy(h.data() + 2 * F + 2 * K, a->lo.data(), 8 * F);
    std::memcpy(h.data() + 3 * F + 2 * K, a->hi.data(), 8 * F);
    double *r = h.data() + 4 * F + 2 * K;
    const chemk_ann_checks &ck = a->checks;
    for (int j = 0; j < ck.n_ratios; ++j) {
        for (int e = 0; e < RAT_E; ++e) {
            r[tr_num + j * RAT_E + e] = ck.ratio_num[j * RAT_E + e];
            r[tr_den + j * RAT_E + e] = ck.ratio_den[j * RAT_E + e];
        }
        r[tr_lo + j] = ck.ratio_lo[j];
        r[tr_hi + j] = ck.ratio_hi[j];
    }
    a->rowtab_stale = true;
    a->generation = next_generation();
    return hipMemcpy(a->normdev, h.data(), 8 * h.size(), hipMemcpyHostToDevice);
}

// The ingest/post tables for the current normalisation (rebuilt after a change).
static hipError_t row_tables(AnnState *a, const DevMech &m, hipStream_t s, const double **ti,
                             const double **tp) {
    const int KM = km_of(a->K);
    if (a->rowtab_stale) {
        hipLaunchKernelGGL(row_tables_kernel, dim3(1), dim3(256), 0, s, m, norm_dev(a), KM, a->rowtab,
                           a->rowtab + ti_size(KM));
        if (hipError_t e = hipGetLastError()) return e;
        a->rowtab_stale = false;
    }
    *ti = a->rowtab;
    *tp = a->rowtab + ti_size(KM);
    return hipSuccess;
}

// Forward of the G = K per-species networks on `rows` packed inputs: the
// first layers of all networks read the same input, so they are one product
// [rows x FPAD] x [FPAD x G pd1]; hidden layer l is a grouped product, network
// g multiplying its column slab g of the previous activations [rows x G pd[l]]
// by its own weights.  Activations of network g sit in columns
// [g pd[l], (g+1) pd[l]).  With two hidden layers or more, the last hidden
// layer's epilogue also applies the one-output layer (EPI_GELU_DOT: BF16
// activations times BF16-rounded output weights, summed in FP32 per 64-column
// half tile), so its activations are never stored, and species_out_kernel
// adds the partial sums and the bias into column k of out [rows x K].  With
// one hidden layer the output layer is one product with a block-diagonal
// [G pd[1] x G] matrix (network g's output weights in block g; its zeros are
// exact in the FP32 sums).
static hipError_t ens_forward(AnnState *a, const uint16_t *X, int rows, float *out, uint16_t *buf0,
                              uint16_t *buf1, hipStream_t s, PhaseTimer *tm) {
    const int G = a->G, L = a->L;
    const bool fuse = a->eW != nullptr;   // L >= 3
    const int S = fuse ? species_slots(a) : 0;
    const uint16_t *in = X;
    uint16_t *bufs[2] = {buf0, buf1};
    for (int l = 0; l < L; ++l) {
        const bool last = l == L - 1;
        const int ph = CHEMK_PHASE_LAYER1 + (l < 3 ? l : 3);
        if (fuse && last) {
            if (tm) tm->begin(ph, s);
            hipLaunchKernelGGL(species_out_kernel, dim3((rows * G + 255) / 256), dim3(256), 0, s, a->eP, S, G,
                               rows, a->eB[l], out);
            if (tm) tm->end(ph, s);
            return hipGetLastError();
        }
        GemmArgs g{};
        g.M = rows;
        g.B = a->Wt[l];
        g.bias = a->eB[l];
        int groups = 1, epi = EPI_BIAS_GELU;
        uint16_t *dst = bufs[l & 1];
        if (l == 0) {
            g.N = G * a->pd[1];
            g.K = FPAD;
            g.A = in;
            g.lda = FPAD;
            g.ldb = FPAD;
        } else if (!last) {
            g.N = a->pd[l + 1];
            g.K = a->pd[l];
            g.A = in;
            g.lda = G * a->pd[l];
            g.ldb = a->pd[l];
            g.gsA = a->pd[l];
            g.gsB = (long long)a->pd[l] * a->pd[l + 1];
            g.gsC = a->pd[l + 1];
            groups = G;
        } else {
            g.N = G;
            g.K = G * a->pd[l];
            g.A = in;
            g.lda = G * a->pd[l];
            g.ldb = G * a->pd[l];
            epi = EPI_BIAS;
        }
        if (last) {
            g.Cf = out;
            g.ldc = G;
        } else if (fuse && l == L - 2) {
            epi = EPI_GELU_DOT;
            g.Zin = a->eW;            // + z pd[L-1] per network (gsC)
            g.Cf = a->eP;
            g.ldc = G * S;
            g.gsCf = S;
        } else {
            g.Cb = dst;
            g.ldcb = G * a->pd[l + 1];
        }
        if (tm) tm->begin(ph, s);
        const hipError_t e = launch_gemm(g, true, true, epi, s, groups);
        if (tm) tm->end(ph, s);
        if (e != hipSuccess) return e;
        in = dst;
    }
    return hipSuccess;
}

#ifndef ENS_CHUNK_MB
#define ENS_CHUNK_MB 3072
#endif
// rows per forward chunk: CHUNK for one network; for an ensemble as many as
// keep the activations of a chunk near ENS_CHUNK_MB MB and the operands' byte
// offsets 31-bit (17,408 rows for the paper's 32 networks of 1600-800-400:
// measured, 192 MB chunks that stay in the memory-side cache ran the forward
// 1.8 times slower, and 48 MB chunks 4.4 times)
static int chunk_rows(const AnnState *a) {
    if (a->G == 1) return CHUNK;
    size_t per = 0, wmax = 0;
    for (int l = 1; l < a->L; ++l) {
        per += 2 * (size_t)a->G * a->pd[l];
        wmax = std::max(wmax, (size_t)a->G * a->pd[l]);
    }
    size_t r = ((size_t)ENS_CHUNK_MB << 20) / per;
    r = std::min(r, (size_t)0x7fffffff / (2 * wmax));
    r = std::max<size_t>(256, r / 256 * 256);
    return (int)std::min<size_t>(r, CHUNK);
}

// forward of `rows` packed inputs X [rows x FPAD] into out [rows x K] (FP32)
static hipError_t mlp_forward(AnnState *a, const uint16_t *X, int rows, float *out, uint16_t *buf0,
                              uint16_t *buf1, hipStream_t s, float **Zsave = nullptr,
                              uint16_t **Asave = nullptr, PhaseTimer *tm = nullptr) {
    if (a->G > 1) return ens_forward(a, X, rows, out, buf0, buf1, s, tm);
    const uint16_t *in = X;
    uint16_t *bufs[2] = {buf0, buf1};
    for (int l = 0; l < a->L; ++l) {
        GemmArgs g{};
        g.M = rows;
        g.N = a->pd[l + 1];
        g.K = a->pd[l];
        g.A = in;
        g.lda = a->pd[l];
        g.B = a->Wt[l];
        g.ldb = a->pd[l];
        g.bias = a->master + a->boff[l];
        const bool last = l == a->L - 1;
        const int ph = CHEMK_PHASE_LAYER1 + (l < 3 ? l : 3);
        if (tm) tm->begin(ph, s);
        hipError_t e;
        if (last) {
            g.Cf = out;
            g.ldc = g.N;
            e = launch_gemm(g, true, true, EPI_BIAS, s);
        } else {
            uint16_t *dst = Asave ? Asave[l + 1] : bufs[l & 1];
            g.Cb = dst;
            g.ldcb = g.N;
            g.Cf = Zsave ? Zsave[l] : nullptr;
            g.ldc = g.N;
            e = launch_gemm(g, true, true, EPI_BIAS_GELU, s);
            in = dst;
        }
        if (tm) tm->end(ph, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static hipError_t ensure_infer(AnnState *a, int64_t n) {
    if (n <= a->cap) return hipSuccess;
    (void)hipFree(a->X);
    (void)hipFree(a->route);
    (void)hipFree(a->h0);
    (void)hipFree(a->out);
    (void)hipFree(a->act[0]);
    (void)hipFree(a->act[1]);
    (void)hipFree(a->eP);
    a->eP = nullptr;
    a->cap = 0;
    int64_t wmax = 0;
    for (int l = 1; l < a->L; ++l) wmax = std::max<int64_t>(wmax, (int64_t)a->G * a->pd[l]);
    const int64_t ch = std::min<int64_t>(n, chunk_rows(a));
    hipError_t e;
    if ((e = hipMalloc(&a->X, sizeof(uint16_t) * n * FPAD)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->route, sizeof(int) * n)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->h0, sizeof(double) * n)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->out, sizeof(float) * n * a->K)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->act[0], sizeof(uint16_t) * ch * wmax)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->act[1], sizeof(uint16_t) * ch * wmax)) != hipSuccess) return e;
    if (a->eW && (e = hipMalloc(&a->eP, sizeof(float) * ch * a->G * species_slots(a))) != hipSuccess) return e;
    a->cap = n;
    a->generation = next_generation();
    return hipSuccess;
}

// Called before a step is enqueued or captured: allocates what the step of n
// cells needs and builds stale tables, so that a captured graph holds no
// allocation and replays the current tables.
hipError_t ann_prepare(AnnState *a, const chemk::DevMech &m, int64_t n, hipStream_t s) {
    hipError_t e = ensure_infer(a, n);
    if (e != hipSuccess) return e;
    const double *ti, *tp;
    return row_tables(a, m, s, &ti, &tp);
}

uint64_t ann_generation(const AnnState *a) { return a ? a->generation : 0; }

static hipError_t launch_post(AnnState *a, const AnnStepArgs &x, const double *tab, hipStream_t s) {
    const DevMech &m = *x.dm;
    const int n = (int)x.n, K = m.K;
    const int grid = (n + POST_CELLS - 1) / POST_CELLS;
    PostChecks ck;
    ck.neg_tol = a->neg_tol;
    ck.adj_max = a->checks.adj_max > 0.0 ? a->checks.adj_max : INFINITY;
    ck.dT_lo = a->checks.dT_lo;
    ck.dT_hi = a->checks.dT_hi;
    return with_km(K, [&](auto km) {
        constexpr int KM = decltype(km)::v;
#define POST_CASE(EE)                                                                             \
    case EE:                                                                                      \
        hipLaunchKernelGGL((post_kernel<EE, KM>), dim3(grid), dim3(POST_CELLS), 0, s, K, n, tab, x.T, \
                           x.Y, a->out, a->route, a->h0, ck, x.project, x.status, x.nsteps,      \
                           x.queue, x.n_routed, x.stats);                                        \
        break;
        switch (m.E) {
            POST_CASE(1)
            POST_CASE(2)
            POST_CASE(3)
            POST_CASE(4)
            POST_CASE(5)
            POST_CASE(6)
            POST_CASE(7)
            POST_CASE(8)
            default:
                return hipErrorInvalidValue;
        }
#undef POST_CASE
        return hipGetLastError();
    });
}

hipError_t ann_enqueue_step(AnnState *a, const AnnStepArgs &x, hipStream_t s) {
    hipError_t e = ensure_infer(a, x.n);
    if (e != hipSuccess) return e;
    const DevMech &m = *x.dm;
    const int n = (int)x.n;
    PhaseTimer *tm = x.timer;
    // counters: stats, routed count, DI queue counter
    hipLaunchKernelGGL(reset_step_kernel, dim3(1), dim3(64), 0, s, x.n_routed, x.counter, x.stats);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // ingest
    if (tm) tm->begin(CHEMK_PHASE_INGEST, s);
    const double *ti, *tp;
    if ((e = row_tables(a, m, s, &ti, &tp)) != hipSuccess) return e;
    if ((e = launch_ingest(m.K, m.E, a->checks.n_ratios, ti, n, x.T, x.p, x.Y, a->X, a->route, a->h0,
                           s)) != hipSuccess)
        return e;
    if (tm) tm->end(CHEMK_PHASE_INGEST, s);
    // MLP in chunks
    if (tm) tm->begin(CHEMK_PHASE_MLP, s);
    const int chunk = chunk_rows(a);
    for (int64_t c0 = 0; c0 < n; c0 += chunk) {
        const int rows = (int)std::min<int64_t>(chunk, n - c0);
        if ((e = mlp_forward(a, a->X + c0 * FPAD, rows, a->out + c0 * a->K, a->act[0], a->act[1], s,
                             nullptr, nullptr, tm)) != hipSuccess)
            return e;
    }
    if (tm) tm->end(CHEMK_PHASE_MLP, s);
    // post
    if (tm) tm->begin(CHEMK_PHASE_POST, s);
    if ((e = launch_post(a, x, tp, s)) != hipSuccess) return e;
    if (tm) tm->end(CHEMK_PHASE_POST, s);
    // DI on the routed cells, the most active stiffness bins first (the
    // ingest's route flags are spent by now: their array takes the ordered
    // queue)
    if (tm) tm->begin(CHEMK_PHASE_FALLBACK, s);
    const int *dq = x.queue;
    if (x.bins > 1) {
        if ((e = launch_binning_list(m, n, x.n_routed, x.queue, x.T, x.p, x.Y, x.dt, x.bins, x.bin, x.hist,
                                     x.offs, a->route, s)) != hipSuccess)
            return e;
        dq = a->route;
    }
    e = launch_di(m, x.di_grid, x.n_routed, dq, x.counter, x.T, x.p, x.Y, x.dt, x.rtol, x.atolY,
                  x.atolT, x.h0_frac, x.max_steps, x.project, x.status, x.nsteps, x.stats,
                  CHEMK_CELL_ROUTED_DI, x.di_kernel, s);
    if (tm) tm->end(CHEMK_PHASE_FALLBACK, s);
    return e;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
AnnState *&ctx_ann(chemk_ctx *c);
chemk::PhaseTimer *ctx_timer(chemk_ctx *c);
int ctx_device(chemk_ctx *c);
int ctx_K(chemk_ctx *c);
void ctx_set_error(const char *msg);
chemk::DevMech ctx_devmech(chemk_ctx *c);

#define ANN_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) {                                                       \
            afail(CHEMK_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));               \
            ctx_set_error(g_ann_err.c_str());                                         \
            return CHEMK_E_HIP;                                                       \
        }                                                                             \
    } while (0)

#define ANN_FAIL(code, ...)                     \
    do {                                        \
        afail(code, __VA_ARGS__);               \
        ctx_set_error(g_ann_err.c_str());       \
        return code;                            \
    } while (0)

static int need_ann(chemk_ctx *c, AnnState **out) {
    if (!c) ANN_FAIL(CHEMK_E_ARG, "null context");
    if (!ctx_ann(c)) ANN_FAIL(CHEMK_E_STATE, "no network: call chemk_ann_create first");
    if (hipSetDevice(ctx_device(c)) != hipSuccess) ANN_FAIL(CHEMK_E_HIP, "hipSetDevice");
    *out = ctx_ann(c);
    return CHEMK_OK;
}

// Sum of the per-output weights of the data term (device [K]): read once,
// checked finite, >= 0 and not all zero.
static int out_weight_sum(chemk_ctx *c, const AnnState *a, const float *w, float *sum) {
    (void)c;
    std::vector<float> h(a->K);
    ANN_TRY(hipMemcpy(h.data(), w, 4 * (size_t)a->K, hipMemcpyDeviceToHost));
    double s = 0.0;
    for (int k = 0; k < a->K; ++k) {
        if (!(h[k] >= 0.f) || !std::isfinite(h[k])) ANN_FAIL(CHEMK_E_ARG, "out_w[%d] = %g is not finite and >= 0", k, h[k]);
        s += h[k];
    }
    if (!(s > 0.0)) ANN_FAIL(CHEMK_E_ARG, "out_w is all zero");
    *sum = (float)s;
    return CHEMK_OK;
}

// Per-species networks train on the data loss alone (each network's own
// output column): no physics terms, no per-output weights.
static int need_plain_loss(AnnState *a, float w_mass, float w_hrr, const float *G, const float *out_w) {
    if (a->G > 1 && (w_mass != 0.f || w_hrr != 0.f || G || out_w))
        ANN_FAIL(CHEMK_E_UNSUPPORTED, "per-species networks train on the data loss alone "
                                      "(no w_mass, w_hrr, G or out_w)");
    return CHEMK_OK;
}

static int create_net(chemk_ctx *c, const int32_t *dims, int32_t L, int G);

extern "C" int chemk_ann_create(chemk_ctx *c, const int32_t *dims, int32_t L) {
    ctx_set_error("");
    if (!c || !dims) ANN_FAIL(CHEMK_E_ARG, "null argument");
    if (L < 1 || L > 16) ANN_FAIL(CHEMK_E_ARG, "n_layers=%d outside [1, 16]", L);
    const int K = ctx_K(c);
    if (dims[L] != K) ANN_FAIL(CHEMK_E_ARG, "dims[L]=%d must be K=%d", dims[L], K);
    return create_net(c, dims, L, 1);
}

extern "C" int chemk_ann_create_species(chemk_ctx *c, const int32_t *dims, int32_t L) {
    ctx_set_error("");
    if (!c || !dims) ANN_FAIL(CHEMK_E_ARG, "null argument");
    if (L < 2 || L > 16) ANN_FAIL(CHEMK_E_ARG, "n_layers=%d outside [2, 16] (one hidden layer at least)", L);
    if (dims[L] != 1) ANN_FAIL(CHEMK_E_ARG, "dims[L]=%d must be 1 (one output per species network)", dims[L]);
    return create_net(c, dims, L, ctx_K(c));
}

static int create_net(chemk_ctx *c, const int32_t *dims, int32_t L, int G) {
    ctx_set_error("");
    const int K = ctx_K(c);
    if (dims[0] != K + 2) ANN_FAIL(CHEMK_E_ARG, "dims[0]=%d must be K+2=%d", dims[0], K + 2);
    if (K + 2 > FPAD) ANN_FAIL(CHEMK_E_UNSUPPORTED, "K+2 > %d inputs", FPAD);
    for (int l = 1; l < L; ++l)
        if (dims[l] < 8 || dims[l] > 8192)
            ANN_FAIL(CHEMK_E_UNSUPPORTED, "hidden width %d outside [8, 8192]", dims[l]);
    if (hipSetDevice(ctx_device(c)) != hipSuccess) ANN_FAIL(CHEMK_E_HIP, "hipSetDevice");
    ann_destroy(ctx_ann(c));
    ctx_ann(c) = nullptr;
    AnnState *a = new AnnState();
    a->K = K;
    a->F = K + 2;
    a->L = L;
    a->G = G;
    a->dims.assign(dims, dims + L + 1);
    // padded widths: the input to the GEMMs' K step, hidden layers to whole
    // 64-column slabs (the padding units have zero weights and biases, so
    // their GELU output and every gradient through them stay zero)
    a->pd = a->dims;
    a->pd[0] = FPAD;
    for (int l = 1; l < L; ++l) a->pd[l] = (dims[l] + 63) / 64 * 64;
    size_t off = 0, pub = 0;
    for (int l = 0; l < L; ++l) {
        a->woff.push_back(off);
        off += (size_t)a->pd[l] * a->pd[l + 1];
        a->boff.push_back(off);
        off += a->pd[l + 1];
        pub += (size_t)a->dims[l] * a->dims[l + 1] + a->dims[l + 1];
    }
    // G networks: master holds G copies of the one-network layout
    a->gstride = off;
    a->nparam = off * G;
    a->npublic = pub * G;
    ctx_ann(c) = a;
    ANN_TRY(hipMalloc(&a->master, 4 * a->nparam));
    ANN_TRY(hipMemset(a->master, 0, 4 * a->nparam));
    ANN_TRY(hipMalloc(&a->grad, 4 * a->nparam));
    ANN_TRY(hipMalloc(&a->m1, 4 * a->nparam));
    ANN_TRY(hipMalloc(&a->m2, 4 * a->nparam));
    ANN_TRY(hipMemset(a->grad, 0, 4 * a->nparam));
    ANN_TRY(hipMemset(a->m1, 0, 4 * a->nparam));
    ANN_TRY(hipMemset(a->m2, 0, 4 * a->nparam));
    if (G == 1) {
        for (int l = 0; l < L; ++l) {
            uint16_t *wt = nullptr, *wb = nullptr;
            ANN_TRY(hipMalloc(&wt, 2 * (size_t)a->pd[l] * a->pd[l + 1]));
            ANN_TRY(hipMalloc(&wb, 2 * (size_t)a->pd[l] * a->pd[l + 1]));
            a->Wt.push_back(wt);
            a->Wb.push_back(wb);
        }
    } else {
        // product operands of the ensemble (see ens_forward): layer 0 one
        // [G pd1 x FPAD] matrix, hidden layers G blocks [pd[l+1] x pd[l]],
        // the output layer block diagonal [G x G pd[L-1]]; biases [G pd[l+1]].
        // For the input gradients of training (ens_fwd_bwd), the untransposed
        // copies: hidden layers G blocks [pd[l] x pd[l+1]], the output layer
        // block diagonal [G pd[L-1] x G]; none for layer 0.
        for (int l = 0; l < L; ++l) {
            const size_t n = l < L - 1 ? (size_t)G * a->pd[l + 1] * a->pd[l] : (size_t)G * G * a->pd[l];
            uint16_t *wt = nullptr, *wb = nullptr;
            float *b = nullptr;
            ANN_TRY(hipMalloc(&wt, 2 * n));
            ANN_TRY(hipMemset(wt, 0, 2 * n));
            if (l > 0) {
                ANN_TRY(hipMalloc(&wb, 2 * n));
                ANN_TRY(hipMemset(wb, 0, 2 * n));
            }
            ANN_TRY(hipMalloc(&b, 4 * (size_t)G * a->pd[l + 1]));
            a->Wt.push_back(wt);
            a->Wb.push_back(wb);
            a->eB.push_back(b);
        }
        if (L >= 3) ANN_TRY(hipMalloc(&a->eW, 4 * (size_t)G * a->pd[L - 1]));
    }
    ANN_TRY(hipMalloc(&a->normdev, 8 * normdev_doubles(a)));
    ANN_TRY(hipMalloc(&a->rowtab, 8 * ROW_TAB_DOUBLES));
    a->mu_x.assign(a->F, 0.0);
    a->sd_x.assign(a->F, 1.0);
    a->mu_y.assign(K, 0.0);
    a->sd_y.assign(K, 1.0);
    a->lo.assign(a->F, -1e300);
    a->hi.assign(a->F, 1e300);
    a->checks = chemk_ann_checks{};
    a->checks.dT_lo = -1e300;
    a->checks.dT_hi = 1e300;
    ANN_TRY(upload_norm(a));
    return CHEMK_OK;
}

extern "C" int chemk_ann_param_count(chemk_ctx *c, int64_t *count) {
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (!count) ANN_FAIL(CHEMK_E_ARG, "null count");
    *count = (int64_t)a->npublic;
    return CHEMK_OK;
}

// public layout <-> internal (layer 0 rows padded from K+2 to FPAD inputs)
// Public layout: per layer W [dims[l] x dims[l+1]] row-major, then b; the
// internal one pads rows to pd[l] and columns to pd[l+1] with zeros.
// With G networks both layouts hold G such vectors one after the other.
static void pub_to_int(const AnnState *a, const float *pub, std::vector<float> &in) {
    in.assign(a->nparam, 0.f);
    size_t p = 0;
    for (int g = 0; g < a->G; ++g) {
        float *base = in.data() + g * a->gstride;
        for (int l = 0; l < a->L; ++l) {
            const int r = a->dims[l], cl = a->dims[l + 1], ld = a->pd[l + 1];
            for (int i = 0; i < r; ++i)
                std::memcpy(base + a->woff[l] + (size_t)i * ld, pub + p + (size_t)i * cl, 4 * cl);
            p += (size_t)r * cl;
            std::memcpy(base + a->boff[l], pub + p, 4 * cl);
            p += cl;
        }
    }
}

static void int_to_pub(const AnnState *a, const float *in, float *pub) {
    size_t p = 0;
    for (int g = 0; g < a->G; ++g) {
        const float *base = in + g * a->gstride;
        for (int l = 0; l < a->L; ++l) {
            const int r = a->dims[l], cl = a->dims[l + 1], ld = a->pd[l + 1];
            for (int i = 0; i < r; ++i)
                std::memcpy(pub + p + (size_t)i * cl, base + a->woff[l] + (size_t)i * ld, 4 * cl);
            p += (size_t)r * cl;
            std::memcpy(pub + p, base + a->boff[l], 4 * cl);
            p += cl;
        }
    }
}

extern "C" int chemk_ann_set_weights(chemk_ctx *c, const float *params, int64_t count) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (!params || count != (int64_t)a->npublic)
        ANN_FAIL(CHEMK_E_ARG, "expected %zu parameters, got %lld", a->npublic, (long long)count);
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(params[i])) ANN_FAIL(CHEMK_E_ARG, "non-finite parameter %lld", (long long)i);
    std::vector<float> in;
    pub_to_int(a, params, in);
    ANN_TRY(hipMemcpy(a->master, in.data(), 4 * a->nparam, hipMemcpyHostToDevice));
    ANN_TRY(refresh_bf16(a, nullptr));
    ANN_TRY(hipDeviceSynchronize());
    a->have_w = true;
    return CHEMK_OK;
}

extern "C" int chemk_ann_get_weights(chemk_ctx *c, float *params, int64_t count) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (!params || count != (int64_t)a->npublic)
        ANN_FAIL(CHEMK_E_ARG, "expected %zu parameters, got %lld", a->npublic, (long long)count);
    std::vector<float> in(a->nparam);
    ANN_TRY(hipDeviceSynchronize());
    ANN_TRY(hipMemcpy(in.data(), a->master, 4 * a->nparam, hipMemcpyDeviceToHost));
    int_to_pub(a, in.data(), params);
    return CHEMK_OK;
}

extern "C" int chemk_ann_set_norm(chemk_ctx *c, const double *mu_x, const double *sd_x,
                                  const double *mu_y, const double *sd_y, double dt) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (!mu_x || !sd_x || !mu_y || !sd_y) ANN_FAIL(CHEMK_E_ARG, "null array");
    if (!(dt > 0) || !std::isfinite(dt)) ANN_FAIL(CHEMK_E_ARG, "dt must be finite and > 0");
    for (int i = 0; i < a->F; ++i)
        if (!std::isfinite(mu_x[i]) || !(sd_x[i] > 0) || !std::isfinite(sd_x[i]))
            ANN_FAIL(CHEMK_E_ARG, "input statistics %d invalid (sd must be > 0)", i);
    for (int i = 0; i < a->K; ++i)
        if (!std::isfinite(mu_y[i]) || !(sd_y[i] > 0) || !std::isfinite(sd_y[i]))
            ANN_FAIL(CHEMK_E_ARG, "output statistics %d invalid (sd must be > 0)", i);
    a->mu_x.assign(mu_x, mu_x + a->F);
    a->sd_x.assign(sd_x, sd_x + a->F);
    a->mu_y.assign(mu_y, mu_y + a->K);
    a->sd_y.assign(sd_y, sd_y + a->K);
    a->dt = dt;
    ANN_TRY(upload_norm(a));
    a->have_norm = true;
    return CHEMK_OK;
}

extern "C" int chemk_ann_get_norm(chemk_ctx *c, double *mu_x, double *sd_x, double *mu_y,
                                  double *sd_y, double *dt) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (!mu_x || !sd_x || !mu_y || !sd_y || !dt) ANN_FAIL(CHEMK_E_ARG, "null array");
    std::memcpy(mu_x, a->mu_x.data(), 8 * a->F);
    std::memcpy(sd_x, a->sd_x.data(), 8 * a->F);
    std::memcpy(mu_y, a->mu_y.data(), 8 * a->K);
    std::memcpy(sd_y, a->sd_y.data(), 8 * a->K);
    *dt = a->dt;
    return CHEMK_OK;
}

extern "C" int chemk_ann_set_envelope(chemk_ctx *c, const double *lo, const double *hi,
                                      double neg_tol) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (!lo || !hi) ANN_FAIL(CHEMK_E_ARG, "null array");
    if (!(neg_tol >= 0)) ANN_FAIL(CHEMK_E_ARG, "neg_tol must be >= 0");
    for (int i = 0; i < a->F; ++i)
        if (!(lo[i] <= hi[i])) ANN_FAIL(CHEMK_E_ARG, "envelope %d: lo > hi", i);
    a->lo.assign(lo, lo + a->F);
    a->hi.assign(hi, hi + a->F);
    a->neg_tol = neg_tol;
    ANN_TRY(upload_norm(a));
    a->have_env = true;
    return CHEMK_OK;
}

extern "C" int chemk_ann_get_envelope(chemk_ctx *c, double *lo, double *hi, double *neg_tol) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (!lo || !hi || !neg_tol) ANN_FAIL(CHEMK_E_ARG, "null array");
    std::memcpy(lo, a->lo.data(), 8 * a->F);
    std::memcpy(hi, a->hi.data(), 8 * a->F);
    *neg_tol = a->neg_tol;
    return CHEMK_OK;
}

extern "C" int chemk_ann_set_checks(chemk_ctx *c, const chemk_ann_checks *ck) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (!ck) ANN_FAIL(CHEMK_E_ARG, "null checks");
    if (std::isnan(ck->adj_max)) ANN_FAIL(CHEMK_E_ARG, "adj_max is NaN");
    if (!(ck->dT_lo <= ck->dT_hi)) ANN_FAIL(CHEMK_E_ARG, "dT window: need dT_lo <= dT_hi");
    if (ck->n_ratios < 0 || ck->n_ratios > CHEMK_MAX_RATIOS)
        ANN_FAIL(CHEMK_E_ARG, "n_ratios=%d outside [0, %d]", ck->n_ratios, CHEMK_MAX_RATIOS);
    const int E = ctx_devmech(c).E;
    for (int j = 0; j < ck->n_ratios; ++j) {
        if (!(ck->ratio_lo[j] <= ck->ratio_hi[j]))
            ANN_FAIL(CHEMK_E_ARG, "ratio window %d: need lo <= hi", j);
        for (int e = 0; e < CHEMK_MAX_ELEMENTS; ++e) {
            const double u = ck->ratio_num[j * CHEMK_MAX_ELEMENTS + e];
            const double d = ck->ratio_den[j * CHEMK_MAX_ELEMENTS + e];
            if (!std::isfinite(u) || !std::isfinite(d))
                ANN_FAIL(CHEMK_E_ARG, "ratio window %d: non-finite coefficient", j);
            if (e >= E && (u != 0.0 || d != 0.0))
                ANN_FAIL(CHEMK_E_ARG, "ratio window %d: coefficient of element %d >= E = %d", j, e, E);
        }
    }
    a->checks = *ck;
    for (int j = ck->n_ratios; j < CHEMK_MAX_RATIOS; ++j) {   // unused windows zeroed
        for (int e = 0; e < CHEMK_MAX_ELEMENTS; ++e)
            a->checks.ratio_num[j * CHEMK_MAX_ELEMENTS + e] = a->checks.ratio_den[j * CHEMK_MAX_ELEMENTS + e] = 0.0;
        a->checks.ratio_lo[j] = a->checks.ratio_hi[j] = 0.0;
    }
    ANN_TRY(upload_norm(a));
    return CHEMK_OK;
}

extern "C" int chemk_ann_get_checks(chemk_ctx *c, chemk_ann_checks *ck) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (!ck) ANN_FAIL(CHEMK_E_ARG, "null checks");
    *ck = a->checks;
    return CHEMK_OK;
}

extern "C" int chemk_ann_fit_envelope(chemk_ctx *c, int64_t n, const double *T, const double *p,
                                      const double *Y, const double *Tn, double q, double widen,
                                      void *stream) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (n < 2 || n > (1ll << 31) - 1) ANN_FAIL(CHEMK_E_ARG, "need 2 <= n < 2^31 states");
    if (!T || !p || !Y) ANN_FAIL(CHEMK_E_ARG, "null array");
    if (!(q >= 0.0 && q < 0.5) || !(widen >= 0.0) || !std::isfinite(widen))
        ANN_FAIL(CHEMK_E_ARG, "need 0 <= q < 0.5 and widen >= 0");
    hipStream_t s = (hipStream_t)stream;
    const DevMech m = ctx_devmech(c);
    EnvSrc src{};
    src.K = a->K;
    src.E = m.E;
    src.F = a->F;
    src.nrat = a->checks.n_ratios;
    src.has_dT = Tn ? 1 : 0;
    src.n = (int)n;
    src.T = T;
    src.p = p;
    src.Y = Y;
    src.Tn = Tn;
    src.Emat = m.Emat;
    for (int i = 0; i < MAX_RATIOS * RAT_E; ++i) {
        src.num[i] = a->checks.ratio_num[i];
        src.den[i] = a->checks.ratio_den[i];
    }
    const int nv = a->F + src.nrat + src.has_dT;
    unsigned long long *mn = nullptr, *mx = nullptr, *cnt = nullptr;
    unsigned int *hist = nullptr;
    double *qlo = nullptr, *qhi = nullptr;
    auto release = [&]() {
        (void)hipFree(mn);
        (void)hipFree(mx);
        (void)hipFree(cnt);
        (void)hipFree(hist);
        (void)hipFree(qlo);
        (void)hipFree(qhi);
    };
    hipError_t e = hipSuccess;
    std::vector<double> hl(nv), hh(nv);
    do {
        if ((e = hipMalloc(&mn, 8 * nv)) || (e = hipMalloc(&mx, 8 * nv)) || (e = hipMalloc(&cnt, 8 * nv)) ||
            (e = hipMalloc(&hist, 4 * (size_t)nv * ENV_BINS)) || (e = hipMalloc(&qlo, 8 * nv)) ||
            (e = hipMalloc(&qhi, 8 * nv)))
            break;
        if ((e = hipMemsetAsync(mn, 0xff, 8 * nv, s)) || (e = hipMemsetAsync(mx, 0, 8 * nv, s)) ||
            (e = hipMemsetAsync(cnt, 0, 8 * nv, s)) ||
            (e = hipMemsetAsync(hist, 0, 4 * (size_t)nv * ENV_BINS, s)))
            break;
        const int gx = (int)std::min<int64_t>(512, (n + 255) / 256);
        hipLaunchKernelGGL(env_range_kernel, dim3(gx, nv), dim3(256), 0, s, src, mn, mx, cnt);
        hipLaunchKernelGGL(env_hist_kernel, dim3(gx, nv), dim3(256), 0, s, src, mn, mx, hist);
        hipLaunchKernelGGL(env_quantile_kernel, dim3((nv + 63) / 64), dim3(64), 0, s, nv, mn, mx, cnt,
                           hist, q, qlo, qhi);
        if ((e = hipGetLastError())) break;
        if ((e = hipMemcpyAsync(hl.data(), qlo, 8 * nv, hipMemcpyDeviceToHost, s)) ||
            (e = hipMemcpyAsync(hh.data(), qhi, 8 * nv, hipMemcpyDeviceToHost, s)))
            break;
        e = hipStreamSynchronize(s);
    } while (false);
    release();
    ANN_TRY(e);
    for (int j = 0; j < nv; ++j)
        if (!std::isfinite(hl[j]) || !std::isfinite(hh[j]))
            ANN_FAIL(CHEMK_E_ARG, "envelope value %d has no finite training value", j);
    auto widened = [&](int j, double &lo, double &hi) {
        const double span = hh[j] - hl[j];
        lo = hl[j] - widen * span;
        hi = hh[j] + widen * span;
    };
    a->lo.resize(a->F);
    a->hi.resize(a->F);
    for (int j = 0; j < a->F; ++j) widened(j, a->lo[j], a->hi[j]);
    // a species absent from a cell (Y_k = 0, Box-Cox -1/lambda) is inside the
    // envelope whatever the training data's lower quantile: the lower tail of
    // a mass fraction is its trace regime, where the feature changes little
    for (int k = 0; k < a->K; ++k) a->lo[k] = std::min(a->lo[k], -1.0 / BCT_LAMBDA);
    for (int r = 0; r < src.nrat; ++r) widened(a->F + r, a->checks.ratio_lo[r], a->checks.ratio_hi[r]);
    if (src.has_dT) widened(a->F + src.nrat, a->checks.dT_lo, a->checks.dT_hi);
    ANN_TRY(upload_norm(a));
    a->have_env = true;
    return CHEMK_OK;
}

extern "C" int chemk_ann_fit_norm(chemk_ctx *c, int64_t n, const double *T, const double *p,
                                  const double *Y, const double *Yn, double dt, double widen,
                                  double neg_tol, void *stream) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (n < 2 || n > (1ll << 31) - 1) ANN_FAIL(CHEMK_E_ARG, "need 2 <= n < 2^31 pairs");
    if (!T || !p || !Y || !Yn) ANN_FAIL(CHEMK_E_ARG, "null array");
    if (!(dt > 0) || !(widen >= 0) || !(neg_tol >= 0)) ANN_FAIL(CHEMK_E_ARG, "bad dt/widen/neg_tol");
    hipStream_t s = (hipStream_t)stream;
    const int K = a->K, F = a->F, nf = 2 * K + 2;
    double *acc = nullptr, *mean = nullptr, *sd = nullptr, *lo = nullptr, *hi = nullptr;
    unsigned long long *mn = nullptr, *mx = nullptr;
    ANN_TRY(hipMalloc(&acc, 8 * nf));
    ANN_TRY(hipMalloc(&mean, 8 * nf));
    ANN_TRY(hipMalloc(&sd, 8 * nf));
    ANN_TRY(hipMalloc(&lo, 8 * nf));
    ANN_TRY(hipMalloc(&hi, 8 * nf));
    ANN_TRY(hipMalloc(&mn, 8 * nf));
    ANN_TRY(hipMalloc(&mx, 8 * nf));
    ANN_TRY(hipMemsetAsync(acc, 0, 8 * nf, s));
    ANN_TRY(hipMemsetAsync(mn, 0xff, 8 * nf, s));
    ANN_TRY(hipMemsetAsync(mx, 0, 8 * nf, s));
    const int gx = (int)std::min<int64_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(stats_kernel, dim3(gx, nf), dim3(256), 0, s, K, (int)n, T, p, Y, Yn, 0,
                       (const double *)nullptr, acc, mn, mx);
    hipLaunchKernelGGL(stats_finish_kernel, dim3(1), dim3(256), 0, s, nf, (int)n, acc, mean, 0);
    ANN_TRY(hipMemsetAsync(acc, 0, 8 * nf, s));
    hipLaunchKernelGGL(stats_kernel, dim3(gx, nf), dim3(256), 0, s, K, (int)n, T, p, Y, Yn, 1,
                       (const double *)mean, acc, mn, mx);
    hipLaunchKernelGGL(stats_finish_kernel, dim3(1), dim3(256), 0, s, nf, (int)n, acc, sd, 1);
    hipLaunchKernelGGL(decode_minmax_kernel, dim3(1), dim3(256), 0, s, nf, mn, mx, lo, hi);
    ANN_TRY(hipGetLastError());
    std::vector<double> hm(nf), hs(nf), hl(nf), hh(nf);
    ANN_TRY(hipMemcpyAsync(hm.data(), mean, 8 * nf, hipMemcpyDeviceToHost, s));
    ANN_TRY(hipMemcpyAsync(hs.data(), sd, 8 * nf, hipMemcpyDeviceToHost, s));
    ANN_TRY(hipMemcpyAsync(hl.data(), lo, 8 * nf, hipMemcpyDeviceToHost, s));
    ANN_TRY(hipMemcpyAsync(hh.data(), hi, 8 * nf, hipMemcpyDeviceToHost, s));
    ANN_TRY(hipStreamSynchronize(s));
    for (auto ptr : {acc, mean, sd, lo, hi}) (void)hipFree(ptr);
    (void)hipFree(mn);
    (void)hipFree(mx);
    for (int j = 0; j < nf; ++j) hs[j] = std::max(hs[j], 1e-12);
    a->mu_x.assign(hm.begin(), hm.begin() + F);
    a->sd_x.assign(hs.begin(), hs.begin() + F);
    a->mu_y.assign(hm.begin() + F, hm.end());
    a->sd_y.assign(hs.begin() + F, hs.end());
    a->lo.resize(F);
    a->hi.resize(F);
    for (int j = 0; j < F; ++j) {
        const double span = hh[j] - hl[j];
        a->lo[j] = hl[j] - widen * span;
        a->hi[j] = hh[j] + widen * span;
    }
    a->neg_tol = neg_tol;
    a->dt = dt;
    ANN_TRY(upload_norm(a));
    a->have_norm = true;
    a->have_env = true;
    return CHEMK_OK;
}

extern "C" int chemk_ann_pack(chemk_ctx *c, int64_t n, const double *T, const double *p,
                              const double *Y, const double *Yn, uint16_t *X, float *Z,
                              void *stream) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (!a->have_norm) ANN_FAIL(CHEMK_E_STATE, "normalisation not set");
    if (n < 0 || n > (1ll << 31) - 1) ANN_FAIL(CHEMK_E_ARG, "bad n");
    if (n == 0) return CHEMK_OK;
    if (!T || !p || !Y || !X || (Z && !Yn)) ANN_FAIL(CHEMK_E_ARG, "null array");
    if (reinterpret_cast<uintptr_t>(X) % 16) ANN_FAIL(CHEMK_E_ARG, "X must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    // reuse the ingest kernel (its route/h0 outputs go to scratch)
    int *route = nullptr;
    double *h0 = nullptr;
    ANN_TRY(hipMalloc(&route, 4 * n));
    ANN_TRY(hipMalloc(&h0, 8 * n));
    const DevMech m = ctx_devmech(c);
    const double *ti, *tp;
    ANN_TRY(row_tables(a, m, s, &ti, &tp));
    ANN_TRY(launch_ingest(m.K, m.E, a->checks.n_ratios, ti, (int)n, T, p, Y, X, route, h0, s));
    if (Z) {
        const int g2 = (int)std::min<int64_t>(8192, (n * a->K + 255) / 256);
        hipLaunchKernelGGL(pack_targets_kernel, dim3(g2), dim3(256), 0, s, a->K, (int)n, Y, Yn,
                           norm_dev(a).mu_y, norm_dev(a).sd_y, Z);
    }
    ANN_TRY(hipGetLastError());
    ANN_TRY(hipStreamSynchronize(s));
    (void)hipFree(route);
    (void)hipFree(h0);
    return CHEMK_OK;
}

extern "C" int chemk_ann_forward_packed(chemk_ctx *c, int64_t n, const uint16_t *X, float *out,
                                        void *stream) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (!a->have_w) ANN_FAIL(CHEMK_E_STATE, "weights not set");
    if (n < 0 || n > (1ll << 31) - 1) ANN_FAIL(CHEMK_E_ARG, "bad n");
    if (n == 0) return CHEMK_OK;
    if (!X || !out) ANN_FAIL(CHEMK_E_ARG, "null array");
    const int chunk = chunk_rows(a);
    ANN_TRY(ensure_infer(a, std::min<int64_t>(n, chunk)));
    hipStream_t s = (hipStream_t)stream;
    PhaseTimer *tm = ctx_timer(c);   // per-layer phases while timing is on
    for (int64_t c0 = 0; c0 < n; c0 += chunk) {
        const int rows = (int)std::min<int64_t>(chunk, n - c0);
        ANN_TRY(mlp_forward(a, X + c0 * FPAD, rows, out + c0 * a->K, a->act[0], a->act[1], s, nullptr,
                            nullptr, tm));
    }
    return CHEMK_OK;
}

// K slices of the weight-gradient product dW = A^T dZ (in x out, K = the
// batch): enough slices that the 128 x 128 output tiles times the slices
// reach about 256 workgroups, each slice at least 64 rows of the batch.
static int dw_split(int in, int out, int B) {
    const int tiles = ((in + 127) / 128) * ((out + 127) / 128);
    int s = 1;
    while (tiles * s < 256 && B % (2 * s) == 0 && B / (2 * s) >= 64) s *= 2;
    return s;
}

static hipError_t ensure_train(AnnState *a, int B) {
    if (B <= a->tB) return hipSuccess;
    (void)hipFree(a->tT[0]);
    (void)hipFree(a->tT[1]);
    a->tT[0] = a->tT[1] = nullptr;
    (void)hipFree(a->tX);
    for (auto p : a->tdZ) (void)hipFree(p);
    a->tdZ.clear();
    (void)hipFree(a->tZt);
    (void)hipFree(a->tGt);
    (void)hipFree(a->tOut);
    (void)hipFree(a->tLoss);
    (void)hipFree(a->tWork);
    a->tWork = nullptr;
    for (auto p : a->tZ) (void)hipFree(p);
    for (size_t i = 1; i < a->tA.size(); ++i) (void)hipFree(a->tA[i]);   // tA[0] aliases tX
    a->tZ.clear();
    a->tA.clear();
    a->tB = 0;
    hipError_t e;
    if ((e = hipMalloc(&a->tX, 2 * (size_t)B * FPAD)) != hipSuccess) return e;
    // widths: G networks side by side (G = 1: one network); pd[L] = 1 per
    // network of an ensemble, K for one network
    const size_t G = a->G;
    for (int l = 0; l < a->L; ++l) {
        uint16_t *d = nullptr;
        if ((e = hipMalloc(&d, 2 * (size_t)B * G * a->pd[l + 1])) != hipSuccess) return e;
        a->tdZ.push_back(d);
    }
    if (!a->side[0]) {
        for (auto &st : a->side)
            if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) return e;
        a->evFork.assign(a->L, nullptr);
        a->evJoin.assign(a->L, nullptr);
        for (int l = 0; l < a->L; ++l)
            if ((e = hipEventCreateWithFlags(&a->evFork[l], hipEventDisableTiming)) != hipSuccess ||
                (e = hipEventCreateWithFlags(&a->evJoin[l], hipEventDisableTiming)) != hipSuccess)
                return e;
    }
    if ((e = hipMalloc(&a->tZt, 4 * (size_t)B * a->K)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->tGt, 4 * (size_t)B * a->K)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->tOut, 4 * (size_t)B * a->K)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->tLoss, 4)) != hipSuccess) return e;
    // per layer (the layers' weight gradients run at once): split-K
    // partials, then the column-sum partials of the bias gradient
    size_t work = 0;
    a->tWoff.assign(a->L, 0);
    // (an ensemble: no split K; the output layer's dense [G pd[L-1] x G]
    // product, whose diagonal blocks are the networks' gradients)
    for (int l = 0; l < a->L; ++l) {
        a->tWoff[l] = work;
        const size_t cs = (size_t)((B + COLSUM_ROWS - 1) / COLSUM_ROWS) * G * a->pd[l + 1];
        if (G == 1) work += (size_t)dw_split(a->pd[l], a->pd[l + 1], B) * a->pd[l] * a->pd[l + 1] + cs;
        else work += (l == a->L - 1 ? G * a->pd[l] * G : 0) + cs;
        work = (work + 63) / 64 * 64;
    }
    if ((e = hipMalloc(&a->tWork, 4 * work)) != hipSuccess) return e;
    for (int l = 0; l < a->L - 1; ++l) {
        float *z = nullptr;
        if ((e = hipMalloc(&z, 4 * (size_t)B * G * a->pd[l + 1])) != hipSuccess) return e;
        a->tZ.push_back(z);
    }
    a->tA.push_back(nullptr);   // layer-0 input is tX
    for (int l = 1; l < a->L; ++l) {
        uint16_t *ap = nullptr;
        if ((e = hipMalloc(&ap, 2 * (size_t)B * G * a->pd[l])) != hipSuccess) return e;
        a->tA.push_back(ap);
    }
    if (G > 1) {
        size_t win = FPAD, wout = 0;
        for (int l = 0; l < a->L; ++l) {
            if (l > 0) win = std::max(win, G * a->pd[l]);
            wout = std::max(wout, G * a->pd[l + 1]);
        }
        if ((e = hipMalloc(&a->tT[0], 2 * (size_t)B * win)) != hipSuccess) return e;
        if ((e = hipMalloc(&a->tT[1], 2 * (size_t)B * wout)) != hipSuccess) return e;
    }
    a->tB = B;
    return hipSuccess;
}

// One training step's forward (saving Z and A), loss and backward on rows
// idx[0..B-1] of (X, Z): the gradient lands in a->grad, the batch loss in sink.

// Loss weights of the physics terms (Eq. 11's W2, W3) and the heat-release
// weights G of the training rows (NULL when w_hrr = 0).
struct PhysLoss {
    const float *G;
    float w_mass, w_hrr;
    const float *out_w;   // per-output weights of the data term (device [K]), NULL = all 1
    float out_wsum;       // their sum
};

// One training step of the G = K per-species networks side by side on rows
// idx[0..B-1] of (X, Z): network k's loss is the mean squared error of its
// own output, column k (the data loss of Eq. 8 for one species).  The
// products are those of ens_forward (first layer one product, hidden layers
// grouped, the output layer block diagonal, without the fused epilogue, since
// the last hidden activations are kept), with pre-activations and activations
// saved; backward: weight gradients of the hidden layers and of the first
// layer (whose input all networks share) as grouped products straight into
// each network's slice of the gradient, the output layer's as one dense
// product whose diagonal blocks are kept, input gradients grouped (dense for
// the output layer), bias gradients as column sums scattered to the slices.
static hipError_t ens_fwd_bwd(AnnState *a, const int32_t *idx, int B, const uint16_t *X, const float *Z,
                              LossSink sink, hipStream_t s) {
    const int K = a->K, L = a->L, G = a->G;
    const size_t gs = a->gstride;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(B), dim3(64), 0, s, idx, B, X, FPAD, Z, K, a->tX, a->tZt);
    a->tA[0] = a->tX;
    hipError_t e;
    for (int l = 0; l < L; ++l) {
        const bool last = l == L - 1;
        GemmArgs g{};
        g.M = B;
        g.B = a->Wt[l];
        g.bias = a->eB[l];
        g.A = a->tA[l];
        int groups = 1, epi = EPI_BIAS_GELU;
        if (l == 0) {
            g.N = G * a->pd[1];
            g.K = FPAD;
            g.lda = FPAD;
            g.ldb = FPAD;
        } else if (!last) {
            g.N = a->pd[l + 1];
            g.K = a->pd[l];
            g.lda = G * a->pd[l];
            g.ldb = a->pd[l];
            g.gsA = a->pd[l];
            g.gsB = (long long)a->pd[l] * a->pd[l + 1];
            g.gsC = a->pd[l + 1];
            g.gsCf = a->pd[l + 1];
            groups = G;
        } else {
            g.N = G;
            g.K = G * a->pd[l];
            g.lda = G * a->pd[l];
            g.ldb = G * a->pd[l];
            epi = EPI_BIAS;
        }
        if (last) {
            g.Cf = a->tOut;
            g.ldc = G;
        } else {
            g.Cf = a->tZ[l];
            g.ldc = G * a->pd[l + 1];
            g.Cb = a->tA[l + 1];
            g.ldcb = G * a->pd[l + 1];
        }
        if ((e = launch_gemm(g, true, true, epi, s, groups)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(mse_kernel, dim3(std::min(1024, (B * K + 255) / 256)), dim3(256), 0, s, a->tOut, a->tZt,
                       B * K, a->tdZ[L - 1], sink, (float)G);
    const int P = (B + COLSUM_ROWS - 1) / COLSUM_ROWS;
    for (int l = L - 1; l >= 0; --l) {
        const bool last = l == L - 1;
        const int in = a->pd[l], out = a->pd[l + 1];   // one network's widths (out = 1 for the output layer)
        const int nall = G * out;                       // columns of dZ_l
        const uint16_t *dZ = a->tdZ[l];
        float *work = a->tWork + a->tWoff[l];
        // weight gradient dW = A^T dZ, contracted over the batch: both
        // operands are first transposed so that the batch is contiguous (the
        // product then loads whole 16-byte chunks without transposing)
        const int wa = l == 0 ? FPAD : G * in;   // columns of this layer's input
        hipLaunchKernelGGL(transpose_bf16_kernel, dim3((wa + TP_TILE - 1) / TP_TILE, (B + TP_TILE - 1) / TP_TILE),
                           dim3(256), 0, s, a->tA[l], B, wa, wa, a->tT[0], B);
        hipLaunchKernelGGL(transpose_bf16_kernel, dim3((nall + TP_TILE - 1) / TP_TILE, (B + TP_TILE - 1) / TP_TILE),
                           dim3(256), 0, s, dZ, B, nall, nall, a->tT[1], B);
        GemmArgs gw{};
        gw.K = B;
        gw.A = a->tT[0];
        gw.lda = B;
        gw.B = a->tT[1];
        gw.ldb = B;
        if (last) {
            gw.M = G * in;
            gw.N = G;
            gw.Cf = work;
            gw.ldc = G;
            if ((e = launch_gemm(gw, true, true, EPI_STORE_F32, s)) != hipSuccess) return e;
            hipLaunchKernelGGL(diag_blocks_kernel, dim3((in * G + 255) / 256), dim3(256), 0, s, work, in, G,
                               a->grad + a->woff[l], gs);
        } else {
            gw.M = in;
            gw.N = out;
            gw.gsA = l == 0 ? 0 : (long long)in * B;
            gw.gsB = (long long)out * B;
            gw.Cf = a->grad + a->woff[l];
            gw.ldc = out;
            gw.gsCf = (long long)gs;
            if ((e = launch_gemm(gw, true, true, EPI_STORE_F32, s, G)) != hipSuccess) return e;
        }
        float *part = last ? work + (size_t)G * in * G : work;
        const int per = nall % 8 == 0 ? 8 : 1;
        hipLaunchKernelGGL(colsum_part_kernel, dim3((nall / per + 63) / 64, P), dim3(64), 0, s, dZ, B, nall, part);
        hipLaunchKernelGGL(colsum_final_kernel, dim3((nall + 255) / 256), dim3(256), 0, s, part, P, nall,
                           a->grad + a->boff[l], out, gs);
        if (l > 0) {
            GemmArgs ga{};
            ga.M = B;
            ga.A = dZ;
            ga.B = a->Wb[l];
            ga.Cb = a->tdZ[l - 1];
            ga.ldcb = G * in;
            ga.Zin = a->tZ[l - 1];
            ga.ldz = G * in;
            int groups = 1;
            if (last) {
                ga.N = G * in;
                ga.K = G;
                ga.lda = G;
                ga.ldb = G;
            } else {
                ga.N = in;
                ga.K = out;
                ga.lda = nall;
                ga.gsA = out;
                ga.ldb = out;
                ga.gsB = (long long)in * out;
                ga.gsC = in;
                groups = G;
            }
            if ((e = launch_gemm(ga, true, true, EPI_GELU_GRAD, s, groups)) != hipSuccess) return e;
        }
    }
    return hipGetLastError();
}

static hipError_t fwd_bwd(AnnState *a, const int32_t *idx, int B, const uint16_t *X, const float *Z,
                          LossSink sink, hipStream_t s, PhysLoss ph = PhysLoss{nullptr, 0.f, 0.f, nullptr, 0.f}) {
    if (a->G > 1) return ens_fwd_bwd(a, idx, B, X, Z, sink, s);
    const int K = a->K, L = a->L;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(B), dim3(64), 0, s, idx, B, X, FPAD, Z, K, a->tX, a->tZt);
    const bool hrr = ph.w_hrr != 0.f && ph.G;
    if (hrr) hipLaunchKernelGGL(gather_g_kernel, dim3(B), dim3(64), 0, s, idx, B, ph.G, K, a->tGt);
    a->tA[0] = a->tX;
    hipError_t e;
    if ((e = mlp_forward(a, a->tX, B, a->tOut, nullptr, nullptr, s, a->tZ.data(), a->tA.data())) != hipSuccess)
        return e;
    if (ph.w_mass != 0.f || hrr || ph.out_w) {
        double S = 0.0;
        for (int k = 0; k < K; ++k) S += a->sd_y[k];
        const NormDev nd = norm_dev(a);
        const float inv_wsum = ph.out_w ? 1.0f / ph.out_wsum : 1.0f / (float)K;
        hipLaunchKernelGGL(phys_loss_kernel, dim3((B + 255) / 256), dim3(256), 0, s, a->tOut, a->tZt,
                           hrr ? a->tGt : nullptr, ph.out_w, inv_wsum, B, K, nd.mu_y, nd.sd_y, (float)(1.0 / S),
                           ph.w_mass, hrr ? ph.w_hrr : 0.f, a->tdZ[L - 1], sink);
    } else {
        hipLaunchKernelGGL(mse_kernel, dim3(std::min(1024, (B * K + 255) / 256)), dim3(256), 0, s, a->tOut,
                           a->tZt, B * K, a->tdZ[L - 1], sink);
    }
    // Backward: the chain of input gradients dZ_{l-1} = (dZ_l W_l^T) * GELU'
    // runs on s.  Under graph capture each layer's weight and bias gradients
    // (which only read dZ_l and the layer's input) fork onto a side stream as
    // soon as dZ_l exists and join s before the caller's Adam step, so that
    // they become parallel branches of the step's graph.  Eager steps keep
    // everything on s (no per-step event traffic, one stream per context).
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if ((e = hipStreamIsCapturing(s, &cs)) != hipSuccess) return e;
    const bool fork = cs == hipStreamCaptureStatusActive;
    for (int l = L - 1; l >= 0; --l) {
        const int in = a->pd[l], out = a->pd[l + 1];
        const uint16_t *dZ = a->tdZ[l];
        hipStream_t sd = fork ? a->side[l % 4] : s;
        if (fork) {
            if ((e = hipEventRecord(a->evFork[l], s)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(sd, a->evFork[l], 0)) != hipSuccess) return e;
        }
        GemmArgs gw{};
        gw.M = in;
        gw.N = out;
        gw.K = B;
        gw.A = a->tA[l];
        gw.lda = in;
        gw.B = dZ;
        gw.ldb = out;
        gw.Cf = a->grad + a->woff[l];
        gw.ldc = out;
        float *work = a->tWork + a->tWoff[l];
        const int split = dw_split(in, out, B);
        if ((e = launch_gemm_splitk(gw, split, work, sd)) != hipSuccess) return e;
        const int P = (B + COLSUM_ROWS - 1) / COLSUM_ROWS;
        float *part = work + (size_t)split * in * out;
        const int per = out % 8 == 0 ? 8 : 1;
        hipLaunchKernelGGL(colsum_part_kernel, dim3((out / per + 63) / 64, P), dim3(64), 0, sd, dZ, B, out, part);
        hipLaunchKernelGGL(colsum_final_kernel, dim3((out + 255) / 256), dim3(256), 0, sd, part, P, out,
                           a->grad + a->boff[l]);
        if (fork && (e = hipEventRecord(a->evJoin[l], sd)) != hipSuccess) return e;
        if (l > 0) {
            GemmArgs ga{};
            ga.M = B;
            ga.N = in;
            ga.K = out;
            ga.A = dZ;
            ga.lda = out;
            ga.B = a->Wb[l];
            ga.ldb = out;
            ga.Cb = a->tdZ[l - 1];
            ga.ldcb = in;
            ga.Zin = a->tZ[l - 1];
            ga.ldz = in;
            if ((e = launch_gemm(ga, true, true, EPI_GELU_GRAD, s)) != hipSuccess) return e;
        }
    }
    if (fork)
        for (int l = 0; l < L; ++l)
            if ((e = hipStreamWaitEvent(s, a->evJoin[l], 0)) != hipSuccess) return e;
    return hipGetLastError();
}

extern "C" int chemk_ann_train_step(chemk_ctx *c, const int32_t *idx, int32_t B, const uint16_t *X,
                                    const float *Z, const float *G, float w_mass, float w_hrr,
                                    const float *out_w, float lr, int32_t update, float *loss, float *grads,
                                    void *stream) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (int r = need_plain_loss(a, w_mass, w_hrr, G, out_w)) return r;
    if (!a->have_w) ANN_FAIL(CHEMK_E_STATE, "weights not set");
    if (!idx || !X || !Z) ANN_FAIL(CHEMK_E_ARG, "null array");
    if (B < 64 || B % 64 != 0 || B > (1 << 20)) ANN_FAIL(CHEMK_E_ARG, "batch %d must be a multiple of 64", B);
    if (!(lr >= 0) || !std::isfinite(lr)) ANN_FAIL(CHEMK_E_ARG, "bad learning rate");
    if (!(w_mass >= 0) || !(w_hrr >= 0) || !std::isfinite(w_mass) || !std::isfinite(w_hrr))
        ANN_FAIL(CHEMK_E_ARG, "loss weights must be finite and >= 0");
    if (w_hrr > 0 && !G) ANN_FAIL(CHEMK_E_ARG, "w_hrr > 0 needs the heat-release weights G");
    ANN_TRY(ensure_train(a, B));
    hipStream_t s = (hipStream_t)stream;
    const int L = a->L;
    hipLaunchKernelGGL(zero_f32_kernel, dim3(1), dim3(64), 0, s, a->tLoss, 1);
    float wsum = 0.f;
    if (out_w)
        if (int r = out_weight_sum(c, a, out_w, &wsum)) return r;
    ANN_TRY(fwd_bwd(a, idx, B, X, Z, LossSink{a->tLoss, nullptr, 1, 1.0f}, s,
                    PhysLoss{G, w_mass, w_hrr, out_w, wsum}));
    if (loss) ANN_TRY(hipMemcpyAsync(loss, a->tLoss, 4, hipMemcpyDeviceToDevice, s));
    if (grads) {   // the public layout: per network, per layer W then b
        size_t p = 0;
        for (int gi = 0; gi < a->G; ++gi) {
            const float *gg = a->grad + gi * a->gstride;
            for (int l = 0; l < L; ++l) {
                const size_t w = (size_t)a->dims[l] * a->dims[l + 1];
                ANN_TRY(hipMemcpy2DAsync(grads + p, 4 * (size_t)a->dims[l + 1], gg + a->woff[l],
                                         4 * (size_t)a->pd[l + 1], 4 * (size_t)a->dims[l + 1], a->dims[l],
                                         hipMemcpyDeviceToDevice, s));
                p += w;
                ANN_TRY(hipMemcpyAsync(grads + p, gg + a->boff[l], 4 * a->dims[l + 1], hipMemcpyDeviceToDevice,
                                       s));
                p += a->dims[l + 1];
            }
        }
    }
    if (update) {
        a->step += 1;
        const double b1 = 0.9, b2 = 0.999;
        const float bc1 = (float)(1.0 / (1.0 - std::pow(b1, (double)a->step)));
        const float bc2 = (float)(1.0 / (1.0 - std::pow(b2, (double)a->step)));
        const int g = (int)std::min<size_t>(4096, (a->nparam + 255) / 256);
        hipLaunchKernelGGL(adam_kernel, dim3(g), dim3(256), 0, s, a->master, a->grad, a->m1, a->m2,
                           (int64_t)a->nparam, lr, (float)b1, (float)b2, 1e-8f, bc1, bc2);
        ANN_TRY(refresh_bf16(a, s));
    }
    return CHEMK_OK;
}

// Held-out loss: the network's forward over the n rows of (X, Z) in chunks,
// the mean squared error added to *acc.
static hipError_t holdout_loss(AnnState *a, int64_t n, const uint16_t *X, const float *Z, float *acc,
                               hipStream_t s) {
    const int chunk = chunk_rows(a);   // the inference buffers hold this many rows
    for (int64_t c0 = 0; c0 < n; c0 += chunk) {
        const int rows = (int)std::min<int64_t>(chunk, n - c0);
        hipError_t e = mlp_forward(a, X + c0 * FPAD, rows, a->out, a->act[0], a->act[1], s);
        if (e != hipSuccess) return e;
        const long long cnt = (long long)rows * a->K;
        hipLaunchKernelGGL(sq_err_kernel, dim3((unsigned)std::min<long long>(1024, (cnt + 255) / 256)),
                           dim3(256), 0, s, a->out, Z + c0 * a->K, cnt, (double)n * a->K, acc);
    }
    return hipGetLastError();
}

extern "C" int chemk_ann_train(chemk_ctx *c, int64_t n, const uint16_t *X, const float *Z,
                               const uint16_t *X_hold, const float *Z_hold, int64_t n_hold,
                               const chemk_train_opts *o, float *epoch_loss, float *hold_loss,
                               void *stream) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (!a->have_w) ANN_FAIL(CHEMK_E_STATE, "weights not set");
    if (!o || !X || !Z) ANN_FAIL(CHEMK_E_ARG, "null argument");
    if (int r = need_plain_loss(a, o->w_mass, o->w_hrr, o->G, o->out_w)) return r;
    const int B = o->batch;
    if (B < 64 || B % 64 != 0 || B > (1 << 20)) ANN_FAIL(CHEMK_E_ARG, "batch %d must be a multiple of 64", B);
    if (n < B || n > (1ll << 31) - 1) ANN_FAIL(CHEMK_E_ARG, "need batch <= n < 2^31 training rows");
    if (o->epochs < 1 || o->epochs > 100000) ANN_FAIL(CHEMK_E_ARG, "epochs=%d outside [1, 1e5]", o->epochs);
    if (o->epoch0 < 0 || o->epoch0 > 100000 ||
        (o->epochs_total != 0 && o->epochs_total < o->epoch0 + o->epochs) || o->epochs_total > 200000)
        ANN_FAIL(CHEMK_E_ARG, "epoch0=%d, epochs=%d and epochs_total=%d do not form a schedule", o->epoch0,
                 o->epochs, o->epochs_total);
    if (!(o->lr0 >= 0) || !(o->lr1 >= 0) || !std::isfinite(o->lr0) || !std::isfinite(o->lr1))
        ANN_FAIL(CHEMK_E_ARG, "bad learning rates");
    if (n_hold < 0 || n_hold > (1ll << 31) - 1 || (n_hold > 0 && (!X_hold || !Z_hold)))
        ANN_FAIL(CHEMK_E_ARG, "bad held-out set");
    if (!(o->w_mass >= 0) || !(o->w_hrr >= 0) || !std::isfinite(o->w_mass) || !std::isfinite(o->w_hrr))
        ANN_FAIL(CHEMK_E_ARG, "loss weights must be finite and >= 0");
    if (o->w_hrr > 0 && !o->G) ANN_FAIL(CHEMK_E_ARG, "w_hrr > 0 needs the heat-release weights G");
    float owsum = 0.f;
    if (o->out_w)
        if (int r = out_weight_sum(c, a, o->out_w, &owsum)) return r;
    if (reinterpret_cast<uintptr_t>(X) % 16 || (X_hold && reinterpret_cast<uintptr_t>(X_hold) % 16))
        ANN_FAIL(CHEMK_E_ARG, "X must be 16-byte aligned");
    hipStream_t s0 = (hipStream_t)stream;
    const int spe = (int)(n / B);
    // this call runs epochs [epoch0, epoch0 + epochs) of a schedule over
    // epochs_total epochs (0: over this call's epochs)
    const long long run = (long long)spe * o->epochs;
    const long long step0 = (long long)spe * o->epoch0;
    const long long total = o->epochs_total > 0 ? (long long)spe * o->epochs_total : step0 + run;
    int half = 1;
    while ((1ll << (2 * half)) < n) ++half;
    // buffers first: nothing is allocated inside the capture
    ANN_TRY(ensure_train(a, B));
    if (n_hold > 0) ANN_TRY(ensure_infer(a, std::min<int64_t>(n_hold, chunk_rows(a))));
    long long *ctl = nullptr;
    int *idx = nullptr;
    float *eloss = nullptr, *hloss = nullptr;
    hipStream_t own = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    auto release = [&]() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (own) (void)hipStreamDestroy(own);
        (void)hipFree(ctl);
        (void)hipFree(idx);
        (void)hipFree(eloss);
        (void)hipFree(hloss);
    };
    hipError_t e = hipSuccess;
    std::vector<float> he(o->epochs, 0.f), hh(o->epochs, 0.f);
    do {
        if ((e = hipMalloc(&ctl, 2 * sizeof(long long))) || (e = hipMalloc(&idx, 4 * (size_t)B)) ||
            (e = hipMalloc(&eloss, 4 * (size_t)o->epochs)) || (e = hipMalloc(&hloss, 4 * (size_t)o->epochs)))
            break;
        hipStream_t s = s0;
        if (o->use_graph && !s) {   // capture needs a stream other than the null stream
            if ((e = hipStreamCreateWithFlags(&own, hipStreamNonBlocking))) break;
            s = own;
        }
        hipLaunchKernelGGL(ctl_init_kernel, dim3(1), dim3(64), 0, s, ctl, step0, (long long)a->step);
        hipLaunchKernelGGL(zero_f32_kernel, dim3((o->epochs + 255) / 256), dim3(256), 0, s, eloss, o->epochs);
        hipLaunchKernelGGL(zero_f32_kernel, dim3((o->epochs + 255) / 256), dim3(256), 0, s, hloss, o->epochs);
        if ((e = hipGetLastError())) break;
        const int gadam = (int)std::min<size_t>(4096, (a->nparam + 255) / 256);
        // one network: the Adam pass writes the BF16 copies itself
        CastTable ct{};
        if (a->G == 1) {
            ct.L = a->L;
            for (int l = 0; l < a->L; ++l) {
                ct.woff[l] = (long long)a->woff[l];
                ct.boff[l] = (long long)a->boff[l];
                ct.in[l] = a->pd[l];
                ct.out[l] = a->pd[l + 1];
                ct.Wt[l] = a->Wt[l];
                ct.Wb[l] = a->Wb[l];
            }
        }
        auto one_step = [&](hipStream_t st) -> hipError_t {
            hipLaunchKernelGGL(batch_index_kernel, dim3((B + 255) / 256), dim3(256), 0, st, ctl, B, spe,
                               (unsigned int)n, half, (unsigned long long)o->seed, idx);
            // the sink indexes epochs by ctl[0] / spe: shifted to this call's first
            hipError_t ee = fwd_bwd(a, idx, B, X, Z, LossSink{eloss - o->epoch0, ctl, spe, 1.0f / (float)spe}, st,
                                    PhysLoss{o->G, o->w_mass, o->w_hrr, o->out_w, owsum});
            if (ee != hipSuccess) return ee;
            hipLaunchKernelGGL(adam_sched_kernel, dim3(gadam), dim3(256), 0, st, a->master, a->grad, a->m1,
                               a->m2, (int64_t)a->nparam, ctl, (double)o->lr0, (double)o->lr1, total, 0.9,
                               0.999, 1e-8f, ct);
            if (a->G > 1 && (ee = refresh_bf16(a, st)) != hipSuccess) return ee;
            hipLaunchKernelGGL(step_end_kernel, dim3(1), dim3(64), 0, st, ctl);
            return hipGetLastError();
        };
        if (o->use_graph) {
            if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal))) break;
            hipError_t ec = one_step(s);
            e = hipStreamEndCapture(s, &graph);
            if (ec) e = ec;
            if (e) break;
            if ((e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0))) break;
        }
        for (int ep = 0; ep < o->epochs && !e; ++ep) {
            for (int b = 0; b < spe && !e; ++b) e = o->use_graph ? hipGraphLaunch(gexec, s) : one_step(s);
            if (!e && n_hold > 0) e = holdout_loss(a, n_hold, X_hold, Z_hold, hloss + ep, s);
        }
        if (e) break;
        if ((e = hipMemcpyAsync(he.data(), eloss, 4 * (size_t)o->epochs, hipMemcpyDeviceToHost, s)) ||
            (e = hipMemcpyAsync(hh.data(), hloss, 4 * (size_t)o->epochs, hipMemcpyDeviceToHost, s)))
            break;
        e = hipStreamSynchronize(s);
    } while (false);
    release();
    ANN_TRY(e);
    a->step += run;
    if (epoch_loss) std::memcpy(epoch_loss, he.data(), 4 * (size_t)o->epochs);
    if (hold_loss) std::memcpy(hold_loss, hh.data(), 4 * (size_t)o->epochs);
    return CHEMK_OK;
}

extern "C" int chemk_ann_hrr_weights(chemk_ctx *c, int64_t n, const double *T, const double *p,
                                     const double *Y, const double *Yn, double dt, double scale_in, float *G,
                                     double *scale_out, void *stream) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (!a->have_norm) ANN_FAIL(CHEMK_E_STATE, "normalisation not set");
    if (n < 1 || n > (1ll << 31) - 1) ANN_FAIL(CHEMK_E_ARG, "bad n");
    if (!T || !p || !Y || !G) ANN_FAIL(CHEMK_E_ARG, "null array");
    if (!(dt > 0) || !std::isfinite(dt)) ANN_FAIL(CHEMK_E_ARG, "dt must be finite and > 0");
    if (!(scale_in >= 0) || !std::isfinite(scale_in)) ANN_FAIL(CHEMK_E_ARG, "bad scale");
    if (scale_in == 0 && !Yn) ANN_FAIL(CHEMK_E_ARG, "the scale from the labels needs Y_next");
    hipStream_t s = (hipStream_t)stream;
    const DevMech m = ctx_devmech(c);
    const NormDev nd = norm_dev(a);
    const int grid = (int)std::min<int64_t>(4096, (n + 255) / 256);
    double scale = scale_in;
    if (scale == 0.0) {
        double *sum2 = nullptr;
        ANN_TRY(hipMalloc(&sum2, 8));
        hipError_t e = hipMemsetAsync(sum2, 0, 8, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(hrr_weights_kernel, dim3(grid), dim3(256), 0, s, m, (int)n, T, p, Y, Yn, dt,
                               nd.sd_y, 0.0, G, sum2);
            e = hipGetLastError();
        }
        double h2 = 0.0;
        if (e == hipSuccess) e = hipMemcpyAsync(&h2, sum2, 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFree(sum2);
        ANN_TRY(e);
        scale = std::sqrt(h2 / (double)n);
        if (!(scale > 0) || !std::isfinite(scale)) ANN_FAIL(CHEMK_E_ARG, "the labels release no heat");
    }
    hipLaunchKernelGGL(hrr_weights_kernel, dim3(grid), dim3(256), 0, s, m, (int)n, T, p, Y, nullptr, dt, nd.sd_y,
                       scale, G, nullptr);
    ANN_TRY(hipGetLastError());
    ANN_TRY(hipStreamSynchronize(s));
    if (scale_out) *scale_out = scale;
    return CHEMK_OK;
}

extern "C" int chemk_ann_reset_optimizer(chemk_ctx *c) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    ANN_TRY(hipMemset(a->m1, 0, 4 * a->nparam));
    ANN_TRY(hipMemset(a->m2, 0, 4 * a->nparam));
    a->step = 0;
    return CHEMK_OK;
}
