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
// 64 x 64 = 4 x 4 MFMA tiles of 16 x 16), K step 64 (two MFMA k-steps),
// double-buffered LDS with a padded row stride.  Workgroups are mapped to
// tiles so that each of the 8 XCDs walks a contiguous range of row blocks
// (the A rows it streams stay in that XCD's L2).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm.h"

namespace chemk {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(4))) float floatx4_t;

constexpr int BM = 128, BN = 128, BK = 64;
constexpr int LDS_LD = BK + 8;   // bf16 elements per LDS row (16-byte pad)
constexpr int NTHREADS = 256;

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
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

// load the (rows x BK) slab of an operand into LDS [rows][LDS_LD]
template <bool KCONT>
__device__ __forceinline__ void load_tile(const uint16_t *__restrict__ G, int ld, int row0,
                                          int rows_total, int k0, int K, uint4 (&reg)[4]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int c = t + q * NTHREADS;   // 0..1023 chunks of 8 bf16
        uint4 v = make_uint4(0, 0, 0, 0);
        if (KCONT) {
            const int r = c >> 3, kc = c & 7;   // 128 rows x 8 chunks
            const int gr = row0 + r, gk = k0 + kc * 8;
            if (gr < rows_total && gk < K)
                v = *reinterpret_cast<const uint4 *>(G + (size_t)gr * ld + gk);
        } else {
            const int k = c >> 4, mc = c & 15;  // 64 k x 16 chunks of 8 rows
            const int gk = k0 + k, gr = row0 + mc * 8;
            if (gk < K && gr < rows_total)
                v = *reinterpret_cast<const uint4 *>(G + (size_t)gk * ld + gr);
        }
        reg[q] = v;
    }
}

template <bool KCONT>
__device__ __forceinline__ void store_tile(uint16_t *S, const uint4 (&reg)[4]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int c = t + q * NTHREADS;
        if (KCONT) {
            const int r = c >> 3, kc = c & 7;
            *reinterpret_cast<uint4 *>(S + r * LDS_LD + kc * 8) = reg[q];
        } else {
            const int k = c >> 4, mc = c & 15;
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&reg[q]);
#pragma unroll
            for (int i = 0; i < 8; ++i) S[(mc * 8 + i) * LDS_LD + k] = e[i];
        }
    }
}

template <bool AK, bool BKc, int EPI>
__global__ void __launch_bounds__(NTHREADS) gemm_bf16_kernel(GemmArgs g) {
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
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

    floatx4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = (floatx4_t){0.f, 0.f, 0.f, 0.f};

    uint4 ra[4], rb[4];
    const int KT = (g.K + BK - 1) / BK;
    load_tile<AK>(g.A, g.lda, m0, g.M, 0, g.K, ra);
    load_tile<BKc>(g.B, g.ldb, n0, g.N, 0, g.K, rb);
    store_tile<AK>(sA[0], ra);
    store_tile<BKc>(sB[0], rb);
    __syncthreads();

    const int fr = lane & 15, fk = (lane >> 4) * 8;
    for (int kt = 0; kt < KT; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < KT) {
            load_tile<AK>(g.A, g.lda, m0, g.M, (kt + 1) * BK, g.K, ra);
            load_tile<BKc>(g.B, g.ldb, n0, g.N, (kt + 1) * BK, g.K, rb);
        }
        const uint16_t *A_ = sA[cur];
        const uint16_t *B_ = sB[cur];
#pragma unroll
        for (int ks = 0; ks < BK; ks += 32) {
            bf16x8_t af[4], bfr[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                af[i] = *reinterpret_cast<const bf16x8_t *>(A_ + (wm + i * 16 + fr) * LDS_LD + ks + fk);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                bfr[j] = *reinterpret_cast<const bf16x8_t *>(B_ + (wn + j * 16 + fr) * LDS_LD + ks + fk);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j],
                                                                        0, 0, 0);
        }
        if (kt + 1 < KT) {
            store_tile<AK>(sA[cur ^ 1], ra);
            store_tile<BKc>(sB[cur ^ 1], rb);
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
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = m0 + wm + i * 16 + (lane & 15);
        if (row >= g.M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = n0 + wn + j * 16 + (lane >> 4) * 4;
            if (col >= g.N) continue;
            const floatx4_t v = acc[i][j];
            const bool full = col + 4 <= g.N;
            float z[4];
            if (EPI == EPI_BIAS_GELU || EPI == EPI_BIAS) {
#pragma unroll
                for (int r = 0; r < 4; ++r) z[r] = v[r] + (col + r < g.N ? g.bias[col + r] : 0.f);
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
                uint16_t o[4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    o[r] = f2bf(EPI == EPI_BIAS_GELU ? gelu_f(z[r]) : z[r] * gelu_grad_f(zin[r]));
                uint16_t *dst = g.Cb + (size_t)row * g.ldcb + col;
                if (full && vcb) {
                    const uint2 pk = make_uint2((uint32_t)o[0] | ((uint32_t)o[1] << 16),
                                                (uint32_t)o[2] | ((uint32_t)o[3] << 16));
                    *reinterpret_cast<uint2 *>(dst) = pk;
                } else {
                    for (int r = 0; r < 4 && col + r < g.N; ++r) dst[r] = o[r];
                }
            }
        }
    }
}

hipError_t launch_gemm(const GemmArgs &g, bool a_kcont, bool b_kcont, int epi, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
    const int grid = ((tiles + 7) / 8) * 8;
#define GEMM_CASE(AKV, BKV, EP)                                                         \
    if (a_kcont == AKV && b_kcont == BKV && epi == EP) {                                \
        hipLaunchKernelGGL((gemm_bf16_kernel<AKV, BKV, EP>), dim3(grid), dim3(NTHREADS), 0, s, g); \
        return hipGetLastError();                                                       \
    }
    GEMM_CASE(true, true, EPI_BIAS_GELU)
    GEMM_CASE(true, true, EPI_BIAS)
    GEMM_CASE(true, true, EPI_GELU_GRAD)
    GEMM_CASE(true, true, EPI_STORE_F32)
    GEMM_CASE(false, false, EPI_STORE_F32)
#undef GEMM_CASE
    return hipErrorInvalidValue;
}

}  // namespace chemk
