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

__device__ __forceinline__ float gelu_f(float x) {
    return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
           x * expf(-0.5f * x * x) * 0.39894228040143268f;
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
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j],
                                                                        0, 0, 0);
        }
        if (kt + 1 < KT) {
            store_tile<AK>(sA[cur ^ 1], ra);
            store_tile<BKc>(sB[cur ^ 1], rb);
        }
        __syncthreads();
    }

    // epilogue: lane holds column (lane & 15) and rows 4*(lane >> 4) + r of each 16x16 tile
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = n0 + wn + j * 16 + (lane & 15);
            if (col >= g.N) continue;
            const float bias = (EPI == EPI_BIAS_GELU || EPI == EPI_BIAS) ? g.bias[col] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                if (row >= g.M) continue;
                const float v = acc[i][j][r];
                if (EPI == EPI_BIAS_GELU) {
                    const float z = v + bias;
                    if (g.Cf) g.Cf[(size_t)row * g.ldc + col] = z;
                    g.Cb[(size_t)row * g.ldcb + col] = f2bf(gelu_f(z));
                } else if (EPI == EPI_BIAS) {
                    g.Cf[(size_t)row * g.ldc + col] = v + bias;
                } else if (EPI == EPI_STORE_F32) {
                    g.Cf[(size_t)row * g.ldc + col] = v;
                } else {   // EPI_GELU_GRAD
                    const float z = g.Zin[(size_t)row * g.ldz + col];
                    g.Cb[(size_t)row * g.ldcb + col] = f2bf(v * gelu_grad_f(z));
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
