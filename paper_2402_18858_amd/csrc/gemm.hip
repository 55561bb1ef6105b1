// gemm.hip -- BF16 GEMM on gfx950 MFMA (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation and fused epilogues, for the MLP that stands in for DI
// (forward pass, and the two backward products of training).
//
// C[M x N] = sum_k A(m, k) B(k, n).  A is "K-contiguous" (A[m*lda + k]) or
// "M-contiguous" (A[k*lda + m]); B is K-contiguous (B[n*ldb + k]) or
// N-contiguous (B[k*ldb + n]).  The forward pass and dA = dZ W^T use the
// K-contiguous form for both operands; dW = A^T dZ uses the other form, and
// the tile loader transposes through LDS.
//
// Tiling: 128 x 128 output tile per 256-thread workgroup (2 x 2 waves, each
// 64 x 64 in MFMA tiles of 16 x 16), K step 64 (two MFMA k-steps),
// double-buffered LDS with a padded row stride.  (The kernel is templated on
// the tile; a 256 x 256 tile with one workgroup per CU measured slower: the
// K loop is bound by the latency of the next slab's global loads.)  Workgroups are mapped to
// tiles so that each of the 8 XCDs walks a contiguous range of row blocks
// (the A rows it streams stay in that XCD's L2).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm.h"

namespace chemk {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(4))) float floatx4_t;

constexpr int NTHREADS = 256;
// bf16 elements per LDS row for a K step of BK (16-byte pad)
template <int BK> constexpr int lds_ld() { return BK + 8; }

typedef __attribute__((ext_vector_type(2))) float floatx2_t;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2_t;

// two FP32 -> packed BF16 (round to nearest even), one v_cvt_pk_bf16_f32
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    const bf16x2_t r = __builtin_convertvector((floatx2_t){lo, hi}, bf16x2_t);
    uint32_t u;
    __builtin_memcpy(&u, &r, 4);
    return u;
}

// erf by Abramowitz & Stegun 7.1.26 (Hastings' rational form): absolute
// error <= 1.5e-7, plus ~1 ulp each from the hardware reciprocal and exp2;
// far below the BF16 spacing of the activations it feeds.  Branch-free,
// ~14 VALU operations against ~30 for the library erff.
__device__ __forceinline__ float erf_as(float x) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
    float poly = fmaf(t, 1.061405429f, -1.453152027f);
    poly = fmaf(t, poly, 1.421413741f);
    poly = fmaf(t, poly, -0.284496736f);
    poly = fmaf(t, poly, 0.254829592f);
    const float e = __builtin_amdgcn_exp2f(-1.44269504088896341f * ax * ax);
    return copysignf(fmaf(-t * poly, e, 1.0f), x);
}

__device__ __forceinline__ float gelu_f(float x) {
    return 0.5f * x * (1.0f + erf_as(x * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erf_as(x * 0.70710678118654752f)) +
           x * __builtin_amdgcn_exp2f(-0.72134752044448170f * x * x) * 0.39894228040143268f;
}

// load the (ROWS x BK) slab of an operand into registers, then LDS [ROWS][LDS_LD]
template <int ROWS, int BK, bool KCONT>
__device__ __forceinline__ void load_tile(const uint16_t *__restrict__ G, int ld, int row0,
                                          int rows_total, int k0, int K,
                                          uint4 (&reg)[ROWS * BK / 8 / NTHREADS]) {
    constexpr int KC = BK / 8;            // chunks of 8 bf16 per row
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < ROWS * BK / 8 / NTHREADS; ++q) {
        const int c = t + q * NTHREADS;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (KCONT) {
            const int r = c / KC, kc = c % KC;   // ROWS rows x KC chunks
            const int gr = row0 + r, gk = k0 + kc * 8;
            if (gr < rows_total && gk < K)
                v = *reinterpret_cast<const uint4 *>(G + (size_t)gr * ld + gk);
        } else {
            constexpr int RC = ROWS / 8;        // chunks of 8 rows per k
            const int k = c / RC, mc = c % RC;  // BK k x RC chunks
            const int gk = k0 + k, gr = row0 + mc * 8;
            if (gk < K && gr < rows_total)
                v = *reinterpret_cast<const uint4 *>(G + (size_t)gk * ld + gr);
        }
        reg[q] = v;
    }
}

template <int ROWS, int BK, bool KCONT>
__device__ __forceinline__ void store_tile(uint16_t *S, const uint4 (&reg)[ROWS * BK / 8 / NTHREADS]) {
    constexpr int KC = BK / 8, LD = lds_ld<BK>();
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < ROWS * BK / 8 / NTHREADS; ++q) {
        const int c = t + q * NTHREADS;
        if (KCONT) {
            const int r = c / KC, kc = c % KC;
            *reinterpret_cast<uint4 *>(S + r * LD + kc * 8) = reg[q];
        } else {
            constexpr int RC = ROWS / 8;
            const int k = c / RC, mc = c % RC;
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&reg[q]);
#pragma unroll
            for (int i = 0; i < 8; ++i) S[(mc * 8 + i) * LD + k] = e[i];
        }
    }
}

// BM x BN output tile per 256-thread workgroup; 2 x 2 waves, each with a
// (BM/2) x (BN/2) tile of TM x TN MFMA tiles of 16 x 16.
template <int BM, int BN, int BK, bool AK, bool BKc, int EPI>
__global__ void __launch_bounds__(NTHREADS) gemm_bf16_kernel(GemmArgs g) {
    constexpr int TM = BM / 32, TN = BN / 32, LDS_LD = lds_ld<BK>();
    __shared__ __attribute__((aligned(16))) uint16_t sA[2][BM * LDS_LD];
    __shared__ __attribute__((aligned(16))) uint16_t sB[2][BN * LDS_LD];

    // XCD-aware tile order: workgroup w runs on XCD (w % 8); XCD x takes the
    // contiguous tile range [x*per, (x+1)*per) in row-block-major order.
    const int mt = (g.M + BM - 1) / BM, nt = (g.N + BN - 1) / BN;
    const int tiles = mt * nt;
    const int per = (tiles + 7) / 8;
    const int w = blockIdx.x;
    const int tile = (w & 7) * per + (w >> 3);
    if (tile >= tiles) return;
    const int tm = tile / nt, tn = tile - tm * nt;
    const int m0 = tm * BM, n0 = tn * BN;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);

    floatx4_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = (floatx4_t){0.f, 0.f, 0.f, 0.f};

    uint4 ra[BM * BK / 8 / NTHREADS], rb[BN * BK / 8 / NTHREADS];
    const int KT = (g.K + BK - 1) / BK;
    load_tile<BM, BK, AK>(g.A, g.lda, m0, g.M, 0, g.K, ra);
    load_tile<BN, BK, BKc>(g.B, g.ldb, n0, g.N, 0, g.K, rb);
    store_tile<BM, BK, AK>(sA[0], ra);
    store_tile<BN, BK, BKc>(sB[0], rb);
    __syncthreads();

    const int fr = lane & 15, fk = (lane >> 4) * 8;
    for (int kt = 0; kt < KT; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < KT) {
            load_tile<BM, BK, AK>(g.A, g.lda, m0, g.M, (kt + 1) * BK, g.K, ra);
            load_tile<BN, BK, BKc>(g.B, g.ldb, n0, g.N, (kt + 1) * BK, g.K, rb);
        }
        const uint16_t *A_ = sA[cur];
        const uint16_t *B_ = sB[cur];
#pragma unroll
        for (int ks = 0; ks < BK; ks += 32) {
            bf16x8_t af[TM], bfr[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                af[i] = *reinterpret_cast<const bf16x8_t *>(A_ + (wm + i * 16 + fr) * LDS_LD + ks + fk);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                bfr[j] = *reinterpret_cast<const bf16x8_t *>(B_ + (wn + j * 16 + fr) * LDS_LD + ks + fk);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j],
                                                                        0, 0, 0);
        }
        if (kt + 1 < KT) {
            store_tile<BM, BK, AK>(sA[cur ^ 1], ra);
            store_tile<BN, BK, BKc>(sB[cur ^ 1], rb);
        }
        __syncthreads();
    }

    // epilogue.  The MFMA computes the 16 x 16 tile transposed (B operand
    // first), so a lane holds row (lane & 15) and the four consecutive
    // columns 4 (lane >> 4) + r of each tile: one 8-byte (BF16) or 16-byte
    // (FP32) access per tile and lane where the leading dimension and the
    // base pointer allow it (they are uniform), element by element otherwise.
    const bool vcf = g.Cf && g.ldc % 4 == 0 && ((uintptr_t)g.Cf & 15) == 0;
    const bool vcb = g.Cb && g.ldcb % 4 == 0 && ((uintptr_t)g.Cb & 7) == 0;
    const bool vz = g.Zin && g.ldz % 4 == 0 && ((uintptr_t)g.Zin & 15) == 0;
    const bool vbias = g.bias && ((uintptr_t)g.bias & 15) == 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int row = m0 + wm + i * 16 + (lane & 15);
        if (row >= g.M) continue;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int col = n0 + wn + j * 16 + (lane >> 4) * 4;
            if (col >= g.N) continue;
            const floatx4_t v = acc[i][j];
            const bool full = col + 4 <= g.N;
            float z[4];
            if (EPI == EPI_BIAS_GELU || EPI == EPI_BIAS) {
                if (full && vbias) {
                    const float4 b = *reinterpret_cast<const float4 *>(g.bias + col);
                    z[0] = v[0] + b.x;
                    z[1] = v[1] + b.y;
                    z[2] = v[2] + b.z;
                    z[3] = v[3] + b.w;
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) z[r] = v[r] + (col + r < g.N ? g.bias[col + r] : 0.f);
                }
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) z[r] = v[r];
            }
            if (EPI == EPI_BIAS || EPI == EPI_STORE_F32 || (EPI == EPI_BIAS_GELU && g.Cf)) {
                float *dst = g.Cf + (size_t)row * g.ldc + col;
                if (full && vcf) {
                    *reinterpret_cast<float4 *>(dst) = make_float4(z[0], z[1], z[2], z[3]);
                } else {
                    for (int r = 0; r < 4 && col + r < g.N; ++r) dst[r] = z[r];
                }
            }
            if (EPI == EPI_BIAS_GELU || EPI == EPI_GELU_GRAD) {
                float zin[4] = {0.f, 0.f, 0.f, 0.f};
                if (EPI == EPI_GELU_GRAD) {
                    const float *zp = g.Zin + (size_t)row * g.ldz + col;
                    if (full && vz) {
                        const float4 q = *reinterpret_cast<const float4 *>(zp);
                        zin[0] = q.x; zin[1] = q.y; zin[2] = q.z; zin[3] = q.w;
                    } else {
                        for (int r = 0; r < 4 && col + r < g.N; ++r) zin[r] = zp[r];
                    }
                }
                float a[4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    a[r] = EPI == EPI_BIAS_GELU ? gelu_f(z[r]) : z[r] * gelu_grad_f(zin[r]);
                const uint2 pk = make_uint2(pack_bf16x2(a[0], a[1]), pack_bf16x2(a[2], a[3]));
                uint16_t *dst = g.Cb + (size_t)row * g.ldcb + col;
                if (full && vcb) {
                    *reinterpret_cast<uint2 *>(dst) = pk;
                } else {
                    const uint16_t o[4] = {(uint16_t)pk.x, (uint16_t)(pk.x >> 16), (uint16_t)pk.y,
                                           (uint16_t)(pk.y >> 16)};
                    for (int r = 0; r < 4 && col + r < g.N; ++r) dst[r] = o[r];
                }
            }
        }
    }
}

hipError_t launch_gemm(const GemmArgs &g, bool a_kcont, bool b_kcont, int epi, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
#define GEMM_CASE(TB, TK, AKV, BKV, EP)                                                 \
    if (a_kcont == AKV && b_kcont == BKV && epi == EP) {                                \
        const int tiles = ((g.M + TB - 1) / TB) * ((g.N + TB - 1) / TB);                \
        const int grid = ((tiles + 7) / 8) * 8;                                         \
        hipLaunchKernelGGL((gemm_bf16_kernel<TB, TB, TK, AKV, BKV, EP>), dim3(grid),     \
                           dim3(NTHREADS), 0, s, g);                                    \
        return hipGetLastError();                                                       \
    }
    GEMM_CASE(128, 64, true, true, EPI_BIAS_GELU)
    GEMM_CASE(128, 64, true, true, EPI_BIAS)
    GEMM_CASE(128, 64, true, true, EPI_GELU_GRAD)
    GEMM_CASE(128, 64, true, true, EPI_STORE_F32)
    GEMM_CASE(128, 64, false, false, EPI_STORE_F32)
#undef GEMM_CASE
    return hipErrorInvalidValue;
}

}  // namespace chemk
