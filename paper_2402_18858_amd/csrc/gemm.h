// gemm.h -- BF16 MFMA GEMM entry (see gemm.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chemk {

enum GemmEpilogue {
    EPI_BIAS_GELU = 0,   // Cb = bf16(gelu(acc + bias)); Cf (optional) = acc + bias
    EPI_BIAS = 1,        // Cf = acc + bias
    EPI_STORE_F32 = 2,   // Cf = acc
    EPI_GELU_GRAD = 3    // Cb = bf16(acc * gelu'(Zin))
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
};

// Any K >= 1 and leading dimensions; operands in whole, 16-byte aligned
// chunks of 8 (K, lda, ldb and the chunked extents multiples of 8) take the
// buffer-load path, others an element-by-element one.  Operands below 2 GiB.
hipError_t launch_gemm(const GemmArgs &g, bool a_kcont, bool b_kcont, int epi, hipStream_t s);

}  // namespace chemk
