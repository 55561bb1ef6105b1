// gemm.h -- BF16 MFMA GEMM entry (see gemm.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chemk {

enum GemmEpilogue {
    EPI_BIAS_GELU = 0,   // Cb = bf16(gelu(acc + bias)); Cf (optional) = acc + bias
    EPI_BIAS = 1,        // Cf = acc + bias
    EPI_STORE_F32 = 2,   // Cf = acc
    EPI_GELU_GRAD = 3,   // Cb = bf16(acc * gelu'(Zin))
    // a = bf16(gelu(acc + bias)) dotted with a weight row: for each output
    // row, each wave-half tile (64 columns) writes sum_c a(row, c) Zin[c] over
    // its columns c < N to Cf[row * ldc + 2 (n0 / 128) + half] (the per-species
    // networks' last hidden layer fused with their one-output layer)
    EPI_GELU_DOT = 4
};

struct GemmArgs {
    int M, N, K;
    const uint16_t *A;
    int lda;
    const uint16_t *B;
    int ldb;
    const float *bias;
    float *Cf;
    int ldc;
    uint16_t *Cb;
    int ldcb;
    const float *Zin;
    int ldz;
    // split K over gridDim.y > 1 slices (launch_gemm_splitk): slice z takes
    // K rows [z K, (z + 1) K) of both operands and writes its partial product
    // to Cf + z * split_stride
    long long split_stride;
    // groups over gridDim.z > 1 (launch_gemm with groups > 1): group z offsets
    // A by z gsA, B by z gsB, bias, Cb and Zin by z gsC, Cf by z gsCf elements
    long long gsA, gsB, gsC, gsCf;
};

// Any K >= 1 and leading dimensions; operands in whole, 16-byte aligned
// chunks of 8 (K, lda, ldb and the chunked extents multiples of 8) take the
// buffer-load path, others an element-by-element one.  Operands below 2 GiB.
// groups > 1 runs that many independent products of the same shape in one
// launch (the per-species layers of an ensemble), group z at the offsets
// gsA, gsB, gsC of GemmArgs; every group's operands must lie within its own
// buffer extents as for a single product.
hipError_t launch_gemm(const GemmArgs &g, bool a_kcont, bool b_kcont, int epi, hipStream_t s, int groups = 1);

// C = A^T B with both operands K-major rows (A [K x M], B [K x N], the
// weight-gradient product of training), FP32 result, K split into `split`
// slices whose partial products go to work [split][M][N] (contiguous, N
// fastest) and are summed in slice order into C (ldc = N).  K must be a
// multiple of split.
hipError_t launch_gemm_splitk(const GemmArgs &g, int split, float *work, hipStream_t s);

}  // namespace chemk
