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

struct NormDev {
    const double *mu_x, *sd_x, *mu_y, *sd_y, *lo, *hi;   // [F], [F], [K], [K], [F], [F]
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
// ingest table: lo, hi, mu_x, 1/sd_x [FPAD each], nasa [7 KM], 1/W [KM]
constexpr int ti_lo = 0, ti_hi = FPAD, ti_mu = 2 * FPAD, ti_sd = 3 * FPAD, ti_nasa = 4 * FPAD;
__host__ __device__ constexpr int ti_invW(int KM) { return 4 * FPAD + 7 * KM; }
__host__ __device__ constexpr int ti_size(int KM) { return 4 * FPAD + 8 * KM; }
// post table: E [E KM], 1/W [KM], a_j (j < 6) [6 KM], mu_y [KM], sd_y [KM]
__host__ __device__ constexpr int tp_invW(int E, int KM) { return E * KM; }
__host__ __device__ constexpr int tp_a(int E, int KM) { return (E + 1) * KM; }
__host__ __device__ constexpr int tp_mu(int E, int KM) { return (E + 7) * KM; }
__host__ __device__ constexpr int tp_sd(int E, int KM) { return (E + 8) * KM; }
__host__ __device__ constexpr int tp_size(int E, int KM) { return (E + 9) * KM; }
constexpr int ROW_TAB_DOUBLES = 4 * FPAD + 8 * 64 + (8 + 9) * 64;

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
    for (int i = threadIdx.x; i < KM; i += blockDim.x) {
        const bool s = i < K;
        ti[ti_invW(KM) + i] = s ? m.invW[i] : 0.0;
        tp[tp_invW(E, KM) + i] = s ? m.invW[i] : 0.0;
        tp[tp_mu(E, KM) + i] = s ? nd.mu_y[i] : 0.0;
        tp[tp_sd(E, KM) + i] = s ? nd.sd_y[i] : 0.0;
        for (int j = 0; j < 6; ++j) tp[tp_a(E, KM) + j * KM + i] = s ? m.nasa[7 * i + j] : 0.0;
        for (int e = 0; e < E; ++e) tp[e * KM + i] = s ? m.Emat[e * K + i] : 0.0;
    }
}

constexpr int POST_CELLS = 64;   // ingest and post: one wave per workgroup

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

// Features (Box-Cox of the K mass fractions, then T and p), z-scored and
// rounded to BF16 into a row of FPAD inputs; the envelope flag (a raw feature
// outside [lo, hi] of the training data, or NaN); the enthalpy h(T, Y) / R
// that the post step conserves.  A group of KP lanes (the power of two >= K,
// equal to the table's KM) takes one cell, lane k its species k, so that the
// species' constants stay in the lane's registers for the whole launch; a
// wave advances 64 / KP cells per iteration, reading their rows of Y and
// writing their rows of X coalesced (lane k: the columns k, k + KP, ...).
constexpr int ING_THREADS = 256;

template <int KP>
__global__ void __launch_bounds__(ING_THREADS) ingest_kernel(int K, int n,
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
    if (sp) {
        lo = tab[ti_lo + k];
        hi = tab[ti_hi + k];
        mu = tab[ti_mu + k];
        isd = tab[ti_sd + k];
        iw = tab[ti_invW(KP) + k];
#pragma unroll
        for (int j = 0; j < 6; ++j) a[j] = tab[ti_nasa + 7 * k + j];
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
        double h = y * iw * hRT;   // zero past K
#pragma unroll
        for (int o = KP / 2; o > 0; o >>= 1) h += __shfl_xor(h, o, 64);
        const bool bad = sp && !((raw >= lo) & (raw <= hi));   // NaN -> outside
        const unsigned long long m = __ballot(bad);
        const bool out = ((m >> (sub * KP)) & gmask) != 0 || !((Tc >= loT) & (Tc <= hiT)) ||
                         !((pc >= lop) & (pc <= hip));
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

// post: y = Y_in + dY (dY = mu + sd * out), two rounds of clipping and the
// element-conserving projection, the admissibility checks, T from h0 by
// Newton; cells that fail any of it are queued for DI and left unchanged.
// The table base plus an opaque uniform zero: loads through it are issued in
// the loop that uses them rather than hoisted out of the round loop, where
// E * KM doubles would not fit in SGPRs.
__device__ __forceinline__ const double *fresh_base(const double *__restrict__ t) {
    int z = 0;
    asm volatile("" : "+s"(z));
    return t + z;
}

template <int E, int KM>
__global__ void __launch_bounds__(POST_CELLS, 2) post_kernel(int K, int n,
                                                             const double *__restrict__ tab,
                                                             double *__restrict__ T,
                                                             double *__restrict__ Y,
                                                             const float *__restrict__ out,
                                                             const int *__restrict__ route,
                                                             const double *__restrict__ h0R,
                                                             double neg_tol, int project,
                                                             int *__restrict__ status,
                                                             int *__restrict__ nsteps,
                                                             int *__restrict__ queue,
                                                             int *__restrict__ n_routed,
                                                             unsigned long long *__restrict__ stats) {
    // Rows go through LDS (stride KM + 1: two-way bank conflicts at most) so
    // that the global reads and writes are coalesced; each lane then holds
    // its cell's row in registers.
    constexpr int ld = KM + 1;
    __shared__ double s_row[POST_CELLS * ld];
    __shared__ int s_keep[POST_CELLS];
    const int base = blockIdx.x * POST_CELLS;
    const int cnt = n - base < POST_CELLS ? n - base : POST_CELLS;
    const int lane = threadIdx.x;
    const bool valid = lane < cnt;
    const int c = valid ? base + lane : base;
    const float invK = 1.0f / (float)K;
    const double *__restrict__ tE = tab;
    rows_to_lds<KM>(Y + (size_t)base * K, cnt, K, invK, s_row, ld);
    __syncthreads();
    double y[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) y[k] = k < K ? s_row[lane * ld + k] : 0.0;
    __syncthreads();
    float *s_out = reinterpret_cast<float *>(s_row);
    rows_to_lds<KM>(out + (size_t)base * K, cnt, K, invK, s_out, ld);
    __syncthreads();
    // element totals of the input state: the projection's target
    double eyin[E];
#pragma unroll
    for (int a = 0; a < E; ++a) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < KM; ++k) acc += tE[a * KM + k] * y[k];
        eyin[a] = acc;
    }
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (k < K) y[k] += tab[tp_mu(E, KM) + k] + tab[tp_sd(E, KM) + k] * (double)s_out[lane * ld + k];
    bool bad = !valid || route[c] != 0;
    // Two rounds of: negative entries set to zero (NaN is kept for the
    // finiteness check), then the projection y <- y - w E^T (E w E^T)^-1
    // (E y - E Y_in), w = max(y, 1e-30), which moves species held at zero by
    // ~1e-30 only.  The second round catches the small species the first
    // correction pushed below zero.  The rounds run on every lane (uniform
    // control flow keeps one copy of the row live); a routed cell's result
    // is discarded, and a singular system leaves y unchanged.
    if (project) {
#pragma unroll 1
        for (int round = 0; round < 2; ++round) {
            double A[E][E], r[E];
#pragma unroll
            for (int a = 0; a < E; ++a) {
                r[a] = -eyin[a];
#pragma unroll
                for (int b = 0; b < E; ++b) A[a][b] = 0.0;
            }
            const double *__restrict__ tE = fresh_base(tab);
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                if (y[k] < 0.0) y[k] = 0.0;
                const double w = y[k] > 1e-30 ? y[k] : 1e-30;
#pragma unroll
                for (int a = 0; a < E; ++a) {
                    const double ew = tE[a * KM + k] * w;
                    r[a] += tE[a * KM + k] * y[k];
#pragma unroll
                    for (int b = 0; b <= a; ++b) A[a][b] += ew * tE[b * KM + k];
                }
            }
#pragma unroll
            for (int a = 0; a < E; ++a)
#pragma unroll
                for (int b = a + 1; b < E; ++b) A[a][b] = A[b][a];
            // Gaussian elimination with partial pivoting
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
#pragma unroll
            for (int a = 0; a < E; ++a) r[a] = ok ? r[a] : 0.0;
            const double *__restrict__ tE2 = fresh_base(tab);
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const double w = y[k] > 1e-30 ? y[k] : 1e-30;
                double acc = 0.0;
#pragma unroll
                for (int a = 0; a < E; ++a) acc += tE2[a * KM + k] * r[a];
                y[k] -= w * acc;   // zero for the padding (E = 0 there)
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (!(y[k] >= -neg_tol) || !isfinite(y[k])) bad = true;
    // Newton on h(T) = h0, as in the property update.  The mixture enthalpy
    // is itself a NASA-7 polynomial in T with coefficients
    // B_j = sum_k (Y_k / W_k) a_jk, built once: each iteration then costs one
    // polynomial instead of one per species.
    double B[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const double w = y[k] * tab[tp_invW(E, KM) + k];
#pragma unroll
        for (int j = 0; j < 6; ++j) B[j] += w * tab[tp_a(E, KM) + j * KM + k];
    }
    double Tn = T[c];
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
        if (st) bad = true;
    }
    if (valid && bad) {
        const int slot = atomicAdd(n_routed, 1);
        queue[slot] = c;
        atomicAdd(&stats[0], 1ull);
    } else if (valid) {
        T[c] = Tn;
        status[c] = 0;
        if (nsteps) nsteps[c] = 0;
    }
    // new rows of the cells that passed; the others keep Y_in
    const bool keep = valid && !bad;
    __syncthreads();
    if (keep) {
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (k < K) s_row[lane * ld + k] = y[k];
    }
    s_keep[lane] = keep ? 1 : 0;
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
        v[r] = s_row[cc * ld + (ii - cc * K)];
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

static hipError_t launch_ingest(int K, const double *tab, int n, const double *T, const double *p,
                                const double *Y, uint16_t *X, int *route, double *h0, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return with_km(K, [&](auto km) {
        constexpr int KP = decltype(km)::v;
        const int64_t groups = ((int64_t)n + 64 / KP - 1) / (64 / KP);
        const int grid = (int)std::min<int64_t>(ingest_resident_grid<KP>(),
                                                (groups + ING_THREADS / 64 - 1) / (ING_THREADS / 64));
        hipLaunchKernelGGL(ingest_kernel<KP>, dim3(grid), dim3(ING_THREADS), 0, s, K, n, tab, T, p, Y, X,
                           route, h0);
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

// MSE on z-scored outputs: loss = mean((out - tgt)^2); dOut = bf16(2 (out - tgt) / count)
__global__ void mse_kernel(const float *__restrict__ out, const float *__restrict__ tgt, int count,
                           uint16_t *dout, float *loss_acc) {
    __shared__ float red[256];
    float s = 0.f;
    const float sc = 2.0f / (float)count;
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
    if (threadIdx.x == 0 && loss_acc) atomicAdd(loss_acc, red[0] / (float)count);
}

// db[o] = sum_b dZ[b][o]  (FP32 accumulation of the BF16 gradient)
__global__ void colsum_kernel(const uint16_t *__restrict__ dZ, int B, int N, float *db) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= N) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += bf2f(dZ[(size_t)b * N + o]);
    db[o] = s;
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
__global__ void cast_layer_kernel(const float *__restrict__ Wm, int in, int out, uint16_t *Wt,
                                  uint16_t *Wb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= in * out) return;
    const int r = i / out, c = i - r * out;
    const uint16_t v = f2bf(Wm[i]);
    Wb[i] = v;
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
    uint16_t *tX = nullptr, *tdZ[2] = {nullptr, nullptr};
    float *tZt = nullptr, *tOut = nullptr, *tLoss = nullptr;
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
    (void)hipFree(a->normdev);
    (void)hipFree(a->rowtab);
    (void)hipFree(a->X);
    (void)hipFree(a->route);
    (void)hipFree(a->h0);
    (void)hipFree(a->out);
    (void)hipFree(a->act[0]);
    (void)hipFree(a->act[1]);
    (void)hipFree(a->tX);
    (void)hipFree(a->tdZ[0]);
    (void)hipFree(a->tdZ[1]);
    (void)hipFree(a->tZt);
    (void)hipFree(a->tOut);
    (void)hipFree(a->tLoss);
    for (auto p : a->tZ) (void)hipFree(p);
    for (size_t i = 1; i < a->tA.size(); ++i) (void)hipFree(a->tA[i]);   // tA[0] aliases tX
    delete a;
}

bool ann_ready(const AnnState *a) { return a && a->have_w && a->have_norm; }
double ann_dt(const AnnState *a) { return a ? a->dt : 0.0; }

static hipError_t refresh_bf16(AnnState *a, hipStream_t s) {
    for (int l = 0; l < a->L; ++l) {
        const int in = a->pd[l], out = a->pd[l + 1];
        hipLaunchKernelGGL(cast_layer_kernel, dim3((in * out + 255) / 256), dim3(256), 0, s,
                           a->master + a->woff[l], in, out, a->Wt[l], a->Wb[l]);
    }
    return hipGetLastError();
}

static NormDev norm_dev(const AnnState *a) {
    const int F = a->F, K = a->K;
    NormDev nd;
    nd.mu_x = a->normdev;
    nd.sd_x = a->normdev + F;
    nd.mu_y = a->normdev + 2 * F;
    nd.sd_y = a->normdev + 2 * F + K;
    nd.lo = a->normdev + 2 * F + 2 * K;
    nd.hi = a->normdev + 3 * F + 2 * K;
    return nd;
}

static hipError_t upload_norm(AnnState *a) {
    const int F = a->F, K = a->K;
    std::vector<double> h(4 * F + 2 * K);
    std::memcpy(h.data(), a->mu_x.data(), 8 * F);
    std::memcpy(h.data() + F, a->sd_x.data(), 8 * F);
    std::memcpy(h.data() + 2 * F, a->mu_y.data(), 8 * K);
    std::memcpy(h.data() + 2 * F + K, a->sd_y.data(), 8 * K);
    std::memcpy(h.data() + 2 * F + 2 * K, a->lo.data(), 8 * F);
    std::memcpy(h.data() + 3 * F + 2 * K, a->hi.data(), 8 * F);
    a->rowtab_stale = true;
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

// forward of `rows` packed inputs X [rows x FPAD] into out [rows x K] (FP32)
static hipError_t mlp_forward(AnnState *a, const uint16_t *X, int rows, float *out, uint16_t *buf0,
                              uint16_t *buf1, hipStream_t s, float **Zsave = nullptr,
                              uint16_t **Asave = nullptr) {
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
    a->cap = 0;
    int wmax = 0;
    for (int l = 1; l < a->L; ++l) wmax = std::max(wmax, a->pd[l]);
    const int64_t ch = std::min<int64_t>(n, CHUNK);
    hipError_t e;
    if ((e = hipMalloc(&a->X, sizeof(uint16_t) * n * FPAD)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->route, sizeof(int) * n)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->h0, sizeof(double) * n)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->out, sizeof(float) * n * a->K)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->act[0], sizeof(uint16_t) * ch * wmax)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->act[1], sizeof(uint16_t) * ch * wmax)) != hipSuccess) return e;
    a->cap = n;
    return hipSuccess;
}

static hipError_t launch_post(AnnState *a, const AnnStepArgs &x, const double *tab, hipStream_t s) {
    const DevMech &m = *x.dm;
    const int n = (int)x.n, K = m.K;
    const int grid = (n + POST_CELLS - 1) / POST_CELLS;
    return with_km(K, [&](auto km) {
        constexpr int KM = decltype(km)::v;
#define POST_CASE(EE)                                                                             \
    case EE:                                                                                      \
        hipLaunchKernelGGL((post_kernel<EE, KM>), dim3(grid), dim3(POST_CELLS), 0, s, K, n, tab, x.T, \
                           x.Y, a->out, a->route, a->h0, a->neg_tol, x.project, x.status,         \
                           x.nsteps, x.queue, x.n_routed, x.stats);                              \
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
    if ((e = launch_ingest(m.K, ti, n, x.T, x.p, x.Y, a->X, a->route, a->h0, s)) != hipSuccess) return e;
    if (tm) tm->end(CHEMK_PHASE_INGEST, s);
    // MLP in chunks
    if (tm) tm->begin(CHEMK_PHASE_MLP, s);
    for (int64_t c0 = 0; c0 < n; c0 += CHUNK) {
        const int rows = (int)std::min<int64_t>(CHUNK, n - c0);
        if ((e = mlp_forward(a, a->X + c0 * FPAD, rows, a->out + c0 * a->K, a->act[0], a->act[1], s)) !=
            hipSuccess)
            return e;
    }
    if (tm) tm->end(CHEMK_PHASE_MLP, s);
    // post
    if (tm) tm->begin(CHEMK_PHASE_POST, s);
    if ((e = launch_post(a, x, tp, s)) != hipSuccess) return e;
    if (tm) tm->end(CHEMK_PHASE_POST, s);
    // DI on the routed cells
    if (tm) tm->begin(CHEMK_PHASE_FALLBACK, s);
    e = launch_di(m, x.di_grid, x.n_routed, x.queue, x.counter, x.T, x.p, x.Y, x.dt, x.rtol, x.atolY,
                  x.atolT, x.h0_frac, x.max_steps, x.project, x.status, x.nsteps, x.stats,
                  CHEMK_CELL_ROUTED_DI, s);
    if (tm) tm->end(CHEMK_PHASE_FALLBACK, s);
    return e;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
AnnState *&ctx_ann(chemk_ctx *c);
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

extern "C" int chemk_ann_create(chemk_ctx *c, const int32_t *dims, int32_t L) {
    ctx_set_error("");
    if (!c || !dims) ANN_FAIL(CHEMK_E_ARG, "null argument");
    const int K = ctx_K(c);
    if (L < 1 || L > 16) ANN_FAIL(CHEMK_E_ARG, "n_layers=%d outside [1, 16]", L);
    if (dims[0] != K + 2) ANN_FAIL(CHEMK_E_ARG, "dims[0]=%d must be K+2=%d", dims[0], K + 2);
    if (dims[L] != K) ANN_FAIL(CHEMK_E_ARG, "dims[L]=%d must be K=%d", dims[L], K);
    if (K + 2 > FPAD) ANN_FAIL(CHEMK_E_UNSUPPORTED, "K+2 > %d inputs", FPAD);
    for (int l = 1; l < L; ++l)
        if (dims[l] < 8 || dims[l] % 64 != 0 || dims[l] > 8192)
            ANN_FAIL(CHEMK_E_UNSUPPORTED, "hidden width %d must be a multiple of 64 in [64, 8192]",
                     dims[l]);
    if (hipSetDevice(ctx_device(c)) != hipSuccess) ANN_FAIL(CHEMK_E_HIP, "hipSetDevice");
    ann_destroy(ctx_ann(c));
    ctx_ann(c) = nullptr;
    AnnState *a = new AnnState();
    a->K = K;
    a->F = K + 2;
    a->L = L;
    a->dims.assign(dims, dims + L + 1);
    a->pd = a->dims;
    a->pd[0] = FPAD;
    size_t off = 0, pub = 0;
    for (int l = 0; l < L; ++l) {
        a->woff.push_back(off);
        off += (size_t)a->pd[l] * a->pd[l + 1];
        a->boff.push_back(off);
        off += a->pd[l + 1];
        pub += (size_t)a->dims[l] * a->dims[l + 1] + a->dims[l + 1];
    }
    a->nparam = off;
    a->npublic = pub;
    ctx_ann(c) = a;
    ANN_TRY(hipMalloc(&a->master, 4 * off));
    ANN_TRY(hipMalloc(&a->grad, 4 * off));
    ANN_TRY(hipMalloc(&a->m1, 4 * off));
    ANN_TRY(hipMalloc(&a->m2, 4 * off));
    ANN_TRY(hipMemset(a->master, 0, 4 * off));
    ANN_TRY(hipMemset(a->grad, 0, 4 * off));
    ANN_TRY(hipMemset(a->m1, 0, 4 * off));
    ANN_TRY(hipMemset(a->m2, 0, 4 * off));
    for (int l = 0; l < L; ++l) {
        uint16_t *wt = nullptr, *wb = nullptr;
        ANN_TRY(hipMalloc(&wt, 2 * (size_t)a->pd[l] * a->pd[l + 1]));
        ANN_TRY(hipMalloc(&wb, 2 * (size_t)a->pd[l] * a->pd[l + 1]));
        a->Wt.push_back(wt);
        a->Wb.push_back(wb);
    }
    ANN_TRY(hipMalloc(&a->normdev, 8 * (4 * a->F + 2 * K)));
    ANN_TRY(hipMalloc(&a->rowtab, 8 * ROW_TAB_DOUBLES));
    a->mu_x.assign(a->F, 0.0);
    a->sd_x.assign(a->F, 1.0);
    a->mu_y.assign(K, 0.0);
    a->sd_y.assign(K, 1.0);
    a->lo.assign(a->F, -1e300);
    a->hi.assign(a->F, 1e300);
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
static void pub_to_int(const AnnState *a, const float *pub, std::vector<float> &in) {
    in.assign(a->nparam, 0.f);
    size_t p = 0;
    for (int l = 0; l < a->L; ++l) {
        const size_t w = (size_t)a->dims[l] * a->dims[l + 1];
        std::memcpy(in.data() + a->woff[l], pub + p, 4 * w);
        p += w;
        std::memcpy(in.data() + a->boff[l], pub + p, 4 * a->dims[l + 1]);
        p += a->dims[l + 1];
    }
}

static void int_to_pub(const AnnState *a, const float *in, float *pub) {
    size_t p = 0;
    for (int l = 0; l < a->L; ++l) {
        const size_t w = (size_t)a->dims[l] * a->dims[l + 1];
        std::memcpy(pub + p, in + a->woff[l], 4 * w);
        p += w;
        std::memcpy(pub + p, in + a->boff[l], 4 * a->dims[l + 1]);
        p += a->dims[l + 1];
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
    ANN_TRY(launch_ingest(m.K, ti, (int)n, T, p, Y, X, route, h0, s));
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
    ANN_TRY(ensure_infer(a, std::min<int64_t>(n, CHUNK)));
    hipStream_t s = (hipStream_t)stream;
    for (int64_t c0 = 0; c0 < n; c0 += CHUNK) {
        const int rows = (int)std::min<int64_t>(CHUNK, n - c0);
        ANN_TRY(mlp_forward(a, X + c0 * FPAD, rows, out + c0 * a->K, a->act[0], a->act[1], s));
    }
    return CHEMK_OK;
}

static hipError_t ensure_train(AnnState *a, int B) {
    if (B <= a->tB) return hipSuccess;
    (void)hipFree(a->tX);
    (void)hipFree(a->tdZ[0]);
    (void)hipFree(a->tdZ[1]);
    (void)hipFree(a->tZt);
    (void)hipFree(a->tOut);
    (void)hipFree(a->tLoss);
    for (auto p : a->tZ) (void)hipFree(p);
    for (size_t i = 1; i < a->tA.size(); ++i) (void)hipFree(a->tA[i]);   // tA[0] aliases tX
    a->tZ.clear();
    a->tA.clear();
    a->tB = 0;
    int wmax = 0;
    for (int l = 0; l <= a->L; ++l) wmax = std::max(wmax, a->pd[l]);
    hipError_t e;
    if ((e = hipMalloc(&a->tX, 2 * (size_t)B * FPAD)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->tdZ[0], 2 * (size_t)B * wmax)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->tdZ[1], 2 * (size_t)B * wmax)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->tZt, 4 * (size_t)B * a->K)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->tOut, 4 * (size_t)B * a->K)) != hipSuccess) return e;
    if ((e = hipMalloc(&a->tLoss, 4)) != hipSuccess) return e;
    for (int l = 0; l < a->L - 1; ++l) {
        float *z = nullptr;
        if ((e = hipMalloc(&z, 4 * (size_t)B * a->pd[l + 1])) != hipSuccess) return e;
        a->tZ.push_back(z);
    }
    a->tA.push_back(nullptr);   // layer-0 input is tX
    for (int l = 1; l < a->L; ++l) {
        uint16_t *ap = nullptr;
        if ((e = hipMalloc(&ap, 2 * (size_t)B * a->pd[l])) != hipSuccess) return e;
        a->tA.push_back(ap);
    }
    a->tB = B;
    return hipSuccess;
}

extern "C" int chemk_ann_train_step(chemk_ctx *c, const int32_t *idx, int32_t B, const uint16_t *X,
                                    const float *Z, float lr, int32_t update, float *loss,
                                    float *grads, void *stream) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    if (!a->have_w) ANN_FAIL(CHEMK_E_STATE, "weights not set");
    if (!idx || !X || !Z) ANN_FAIL(CHEMK_E_ARG, "null array");
    if (B < 64 || B % 64 != 0 || B > (1 << 20)) ANN_FAIL(CHEMK_E_ARG, "batch %d must be a multiple of 64", B);
    if (!(lr >= 0) || !std::isfinite(lr)) ANN_FAIL(CHEMK_E_ARG, "bad learning rate");
    ANN_TRY(ensure_train(a, B));
    hipStream_t s = (hipStream_t)stream;
    const int K = a->K, L = a->L;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(B), dim3(64), 0, s, idx, B, X, FPAD, Z, K, a->tX, a->tZt);
    a->tA[0] = a->tX;
    ANN_TRY(hipMemsetAsync(a->tLoss, 0, 4, s));
    // forward with saved pre-activations and activations
    ANN_TRY(mlp_forward(a, a->tX, B, a->tOut, nullptr, nullptr, s, a->tZ.data(), a->tA.data()));
    // loss and output gradient
    hipLaunchKernelGGL(mse_kernel, dim3(std::min(1024, (B * K + 255) / 256)), dim3(256), 0, s, a->tOut,
                       a->tZt, B * K, a->tdZ[0], a->tLoss);
    // backward
    int cur = 0;
    for (int l = L - 1; l >= 0; --l) {
        const int in = a->pd[l], out = a->pd[l + 1];
        const uint16_t *dZ = a->tdZ[cur];
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
        ANN_TRY(launch_gemm(gw, false, false, EPI_STORE_F32, s));
        hipLaunchKernelGGL(colsum_kernel, dim3((out + 255) / 256), dim3(256), 0, s, dZ, B, out,
                           a->grad + a->boff[l]);
        if (l > 0) {
            GemmArgs ga{};
            ga.M = B;
            ga.N = in;
            ga.K = out;
            ga.A = dZ;
            ga.lda = out;
            ga.B = a->Wb[l];
            ga.ldb = out;
            ga.Cb = a->tdZ[cur ^ 1];
            ga.ldcb = in;
            ga.Zin = a->tZ[l - 1];
            ga.ldz = in;
            ANN_TRY(launch_gemm(ga, true, true, EPI_GELU_GRAD, s));
            cur ^= 1;
        }
    }
    ANN_TRY(hipGetLastError());
    if (loss) ANN_TRY(hipMemcpyAsync(loss, a->tLoss, 4, hipMemcpyDeviceToDevice, s));
    if (grads) {
        size_t p = 0;
        for (int l = 0; l < L; ++l) {
            const size_t w = (size_t)a->dims[l] * a->dims[l + 1];
            ANN_TRY(hipMemcpyAsync(grads + p, a->grad + a->woff[l], 4 * w, hipMemcpyDeviceToDevice, s));
            p += w;
            ANN_TRY(hipMemcpyAsync(grads + p, a->grad + a->boff[l], 4 * a->dims[l + 1],
                                   hipMemcpyDeviceToDevice, s));
            p += a->dims[l + 1];
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

extern "C" int chemk_ann_reset_optimizer(chemk_ctx *c) {
    ctx_set_error("");
    AnnState *a;
    if (int r = need_ann(c, &a)) return r;
    ANN_TRY(hipMemset(a->m1, 0, 4 * a->nparam));
    ANN_TRY(hipMemset(a->m2, 0, 4 * a->nparam));
    a->step = 0;
    return CHEMK_OK;
}
