// gemm.hip -- BF16 GEMM on gfx950 MFMA (v_mfma_f32_32x32x16_bf16) with FP32
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
// 64 x 64 in MFMA tiles of 32 x 32), K step 64 (four MFMA k-steps).  Two
// kernels:
//  * forward layers whose slab count is one the networks have (1, 4, 8, 16;
//    13 and 25 for the per-species networks): the slabs go from global
//    memory straight into LDS (buffer loads with an LDS destination), into
//    unpadded rows with a swizzled chunk order.  1, 8, 13, 16 and 25 slabs
//    use a single LDS stage shared with the output staging (37 KB,
//    four workgroups per CU, which hide each other's slab loads); 4 slabs
//    (the last layer) use two stages and prefetch;
//  * everything else (training products, transposing loads, other K): two
//    LDS stages, and a ring of registers holds the next slabs (buffer loads,
//    which read zeros past an operand's edge, so no load sits behind a
//    branch); the tile is stored into LDS rows with a 16-byte pad.
// Forward BF16 outputs leave through LDS so that each store instruction
// writes whole 128-byte row segments.  Workgroups are mapped to tiles so that
// each of the 8 XCDs walks a contiguous range of row blocks (the A rows it
// streams stay in that XCD's L2).  Measured alternatives that lost: a 256 x
// 256 tile with one workgroup per CU, a two-group ping-pong schedule, deeper
// register rings; the 16 x 16 x 32 MFMA needs twice the independent
// accumulations in flight for the same rate.  The first layer's time is the
// VALU work of its GELU epilogue, hence the reciprocal-free GELU below.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "gemm.h"

namespace chemk {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(4))) float floatx4_t;
typedef __attribute__((ext_vector_type(16))) float floatx16_t;

// One MFMA: a 32 x 32 x 16 product, B operand first, so that the result is
// the transposed tile (see the epilogue).  (The 16 x 16 x 32 form does the
// same work in half the output; measured on gfx950 it needs some 32
// independent accumulations in flight per SIMD to reach the rate this one
// reaches with 8.)
__device__ __forceinline__ floatx16_t mfma32(const bf16x8_t &b, const bf16x8_t &a, const floatx16_t &c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(b, a, c, 0, 0, 0);
}

constexpr int NTHREADS = 256;


// bf16 elements per LDS row for a K step of BK (16-byte pad)
template <int BK> constexpr int lds_ld() { return BK + 8; }

// the group's operands of a grouped launch (gridDim.z > 1): the per-species
// networks' hidden layers, network z multiplying its own column slab of the
// activations by its own weights
__device__ __forceinline__ void group_offsets(GemmArgs &g) {
    if (gridDim.z > 1) {
        const long long z = blockIdx.z;
        g.A += z * g.gsA;
        g.B += z * g.gsB;
        const long long c = z * g.gsC;
        if (g.bias) g.bias += c;
        if (g.Cf) g.Cf += z * g.gsCf;
        if (g.Cb) g.Cb += c;
        if (g.Zin) g.Zin += c;
    }
}

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

// Forward GELU(x) = x Phi(x) with Phi(x) = 1/2 + x P(x^2) on |x| <= 4.5 and
// x clamped to +-4.5 outside (where Phi is within 3.4e-6 of 0 or 1).  P is a
// degree-11 polynomial in t = x^2 - 8.1 (centred, so that its terms do not
// cancel in FP32), fitted near-minimax to the error function on the clamped
// range: |Phi error| <= 2.1e-7, GELU absolute error <= 5.7e-7 for |x| <= 3
// and relative error <= 3.6e-6 for x > 0.05, so that the BF16 activations
// it feeds round as those of the exact GELU do in all but about 2.5 % of
// cases, each one BF16 step apart.  Cost: a clamp and thirteen FMAs, no
// reciprocal or exponential.  +-inf gives +-inf, NaN gives NaN.
__device__ __forceinline__ float gelu_f(float x) {
    const float xc = __builtin_amdgcn_fmed3f(x, -4.5f, 4.5f);   // NaN leaves through the final x *
    const float t = fmaf(xc, xc, -8.1f);
    float p = fmaf(t, -2.815799249853996e-15f, 1.4671269299264267e-13f);
    p = fmaf(t, p, -3.6212595422302485e-12f);
    p = fmaf(t, p, 6.798075297131945e-11f);
    p = fmaf(t, p, -1.262795756851176e-09f);
    p = fmaf(t, p, 2.2716244885145898e-08f);
    p = fmaf(t, p, -3.6728903296534554e-07f);
    p = fmaf(t, p, 5.314901500241831e-06f);
    p = fmaf(t, p, -6.984318315517157e-05f);
    p = fmaf(t, p, 0.0008526599849574268f);
    p = fmaf(t, p, -0.01036753784865141f);
    p = fmaf(t, p, 0.174904465675354f);
    return x * fmaf(xc, p, 0.5f);
}

__device__ __forceinline__ float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erf_as(x * 0.70710678118654752f)) +
           x * __builtin_amdgcn_exp2f(-0.72134752044448170f * x * x) * 0.39894228040143268f;
}

// Workgroup barrier that orders LDS only: unlike __syncthreads() it does not
// wait for outstanding global loads, which are the slabs in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

typedef __attribute__((ext_vector_type(4))) unsigned int u32x4_t;


// Buffer resource over one operand: raw buffer loads return zero for offsets
// past num_records, which is how the tile loader handles the edges.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t operand_rsrc(const uint16_t *p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, 0, (int)bytes, 0x00020000);
}

// Up to 8 consecutive elements of G from element offset `at` (nvalid of
// them, zeros after), element by element: for operands whose chunks are not
// 16-byte aligned or run past the operand's edge.
__device__ __forceinline__ uint4 load_chunk_slow(const uint16_t *G, size_t at, int nvalid) {
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if (e < nvalid) w[e >> 1] |= (uint32_t)G[at + e] << (16 * (e & 1));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// load the (ROWS x BK) slab of an operand into registers (then LDS
// [ROWS][LDS_LD]), shared by the NTHREADS threads t of a loading group.  Where the operands are stored in whole 16-byte chunks
// (VEC, chosen by the host), every chunk is one buffer load, and a chunk outside the
// operand gets an offset past the buffer's end and so reads as zeros: no
// branch surrounds a load, so the compiler can wait for one slab while later
// slabs stay in flight.  Other shapes (small training layers) load element by
// element.  (The host guarantees operands below 2 GiB.)
template <int ROWS, int BK, bool KCONT, bool VEC>
__device__ __forceinline__ void load_tile(__amdgpu_buffer_rsrc_t rs, const uint16_t *G,
                                          int ld, int row0, int rows_total, int k0, int K,
                                          uint4 (&reg)[ROWS * BK / 8 / NTHREADS], int t) {
    constexpr int KC = BK / 8;            // chunks of 8 bf16 per row
#pragma unroll
    for (int q = 0; q < ROWS * BK / 8 / NTHREADS; ++q) {
        const int c = t + q * NTHREADS;
        int gr, gk;
        size_t at;
        int nvalid;
        if (KCONT) {
            const int r = c / KC, kc = c % KC;   // ROWS rows x KC chunks
            gr = row0 + r;
            gk = k0 + kc * 8;
            at = (size_t)gr * ld + gk;
            nvalid = gr < rows_total ? min(8, K - gk) : 0;
        } else {
            constexpr int RC = ROWS / 8;        // chunks of 8 rows per k
            const int k = c / RC, mc = c % RC;  // BK k x RC chunks
            gk = k0 + k;
            gr = row0 + mc * 8;
            at = (size_t)gk * ld + gr;
            nvalid = gk < K ? min(8, rows_total - gr) : 0;
        }
        if constexpr (VEC) {
            const int off = nvalid > 0 ? (int)(2 * at) : 0x7fffffff;
            const u32x4_t v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
            reg[q] = make_uint4(v.x, v.y, v.z, v.w);
        } else {
            reg[q] = load_chunk_slow(G, at, nvalid);
        }
    }
}

template <int ROWS, int BK, bool KCONT>
__device__ __forceinline__ void store_tile(uint16_t *S, const uint4 (&reg)[ROWS * BK / 8 / NTHREADS],
                                           int t) {
    constexpr int KC = BK / 8, LD = lds_ld<BK>();
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

// Epilogue of a BM x BN tile whose wave (wm, wn) holds the TM x TN MFMA
// tiles acc of 32 x 32.  The MFMA computes each tile transposed (B operand
// first), so a lane holds row (lane & 31) and, for q = 0..3, the four
// consecutive columns 8 q + 4 (lane >> 5) + r: one 8-byte (BF16) or 16-byte
// (FP32) access per quad and lane where the leading dimension and the base
// pointer allow it (they are uniform), element by element otherwise.
template <int BM, int BN, int EPI, int TM = BM / 64, int TN = BN / 64>
__device__ __forceinline__ void epilogue(const GemmArgs &g, const floatx16_t (&acc)[TM][TN], int m0,
                                         int n0, int wm, int wn, int lane, uint16_t *stage) {
    const bool vcf = g.Cf && g.ldc % 4 == 0 && ((uintptr_t)g.Cf & 15) == 0;
    const bool vcb = g.Cb && g.ldcb % 4 == 0 && ((uintptr_t)g.Cb & 7) == 0;
    const bool vz = g.Zin && g.ldz % 4 == 0 && ((uintptr_t)g.Zin & 15) == 0;
    const bool vbias = g.bias && ((uintptr_t)g.bias & 15) == 0;
    const int lr = lane & 31, lc = (lane >> 5) * 4;
    // The last hidden layer of the per-species networks fused with their
    // output layer: the activations never leave the registers.  Lane l holds
    // rows wm + 32 i + (l % 32) and columns wn + 32 j + 8 q + 4 (l / 32) + r;
    // each lane sums its columns' a Zin products, lanes l and l + 32 (the same
    // rows) add theirs, and the wave's 64 rows get one partial each.  N is a
    // multiple of 4, so a quad of columns is inside or outside as a whole.
    if constexpr (EPI == EPI_GELU_DOT) {
        const int slot = 2 * (n0 / BN) + (wn ? 1 : 0);
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            float sum = 0.f;
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int col = n0 + wn + j * 32 + q * 8 + lc;
                    if (col < g.N) {
                        const float4 b = *reinterpret_cast<const float4 *>(g.bias + col);
                        const float4 w = *reinterpret_cast<const float4 *>(g.Zin + col);
                        const floatx16_t &v = acc[i][j];
                        const uint32_t p0 = pack_bf16x2(gelu_f(v[4 * q] + b.x), gelu_f(v[4 * q + 1] + b.y));
                        const uint32_t p1 = pack_bf16x2(gelu_f(v[4 * q + 2] + b.z), gelu_f(v[4 * q + 3] + b.w));
                        sum = fmaf(__uint_as_float(p0 << 16), w.x, sum);
                        sum = fmaf(__uint_as_float(p0 & 0xffff0000u), w.y, sum);
                        sum = fmaf(__uint_as_float(p1 << 16), w.z, sum);
                        sum = fmaf(__uint_as_float(p1 & 0xffff0000u), w.w, sum);
                    }
                }
            sum += __shfl_xor(sum, 32, 64);
            const int row = m0 + wm + i * 32 + lr;
            if (lane < 32 && row < g.M) g.Cf[(size_t)row * g.ldc + slot] = sum;
        }
        return;
    }
    // Forward BF16-only layers on a whole tile: the wave's (BM/2) x (BN/2)
    // output goes through its LDS staging area (rows of BN/2 + 8 elements) so
    // that each global store instruction writes whole 128-byte row segments
    // (eight of them) instead of 16 bytes in each of 32 rows.  The caller has
    // made the staging area free with a workgroup barrier; the condition is
    // uniform over the workgroup.
    if constexpr (EPI == EPI_BIAS_GELU) {
        constexpr int WR = BM / 2, WC = BN / 2, SLD = WC + 8, CH = WC / 8;
        if (m0 + BM <= g.M && n0 + BN <= g.N && vbias && !g.Cf && g.Cb && g.ldcb % 8 == 0 &&
            ((uintptr_t)g.Cb & 15) == 0) {
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = j * 32 + q * 8 + lc;
                    const float4 bj = *reinterpret_cast<const float4 *>(g.bias + n0 + wn + c);
#pragma unroll
                    for (int i = 0; i < TM; ++i) {
                        const floatx16_t &v = acc[i][j];
                        *reinterpret_cast<uint2 *>(stage + (i * 32 + lr) * SLD + c) =
                            make_uint2(pack_bf16x2(gelu_f(v[4 * q] + bj.x), gelu_f(v[4 * q + 1] + bj.y)),
                                       pack_bf16x2(gelu_f(v[4 * q + 2] + bj.z), gelu_f(v[4 * q + 3] + bj.w)));
                    }
                }
            // the wave reads back only what it wrote: a wave-scope LDS fence
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
#pragma unroll
            for (int r = 0; r < WR * CH / 64; ++r) {
                const int ck = r * 64 + lane;           // chunk of 8 elements: row ck / CH
                const int row = ck / CH, c8 = (ck % CH) * 8;
                const uint4 w = *reinterpret_cast<const uint4 *>(stage + row * SLD + c8);
                *reinterpret_cast<uint4 *>(g.Cb + (size_t)(m0 + wm + row) * g.ldcb + n0 + wn + c8) = w;
            }
            return;
        }
    }
    // Forward layers on a tile wholly inside the output with aligned operands
    // (the usual case; the condition is uniform): no bounds tests, one vector
    // bias load, store and (BF16) packed store per quad and lane.
    if constexpr (EPI == EPI_BIAS_GELU || EPI == EPI_BIAS) {
        if (m0 + BM <= g.M && n0 + BN <= g.N && vbias && (EPI == EPI_BIAS ? vcf : vcb && (!g.Cf || vcf))) {
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int col = n0 + wn + j * 32 + q * 8 + lc;
                    const float4 bj = *reinterpret_cast<const float4 *>(g.bias + col);
#pragma unroll
                    for (int i = 0; i < TM; ++i) {
                        const int row = m0 + wm + i * 32 + lr;
                        const floatx16_t &v = acc[i][j];
                        const float z0 = v[4 * q] + bj.x, z1 = v[4 * q + 1] + bj.y;
                        const float z2 = v[4 * q + 2] + bj.z, z3 = v[4 * q + 3] + bj.w;
                        if (EPI == EPI_BIAS || g.Cf)
                            *reinterpret_cast<float4 *>(g.Cf + (size_t)row * g.ldc + col) =
                                make_float4(z0, z1, z2, z3);
                        if constexpr (EPI == EPI_BIAS_GELU)
                            *reinterpret_cast<uint2 *>(g.Cb + (size_t)row * g.ldcb + col) =
                                make_uint2(pack_bf16x2(gelu_f(z0), gelu_f(z1)),
                                           pack_bf16x2(gelu_f(z2), gelu_f(z3)));
                    }
                }
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int row = m0 + wm + i * 32 + lr;
        if (row >= g.M) continue;
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int col = n0 + wn + j * 32 + q * 8 + lc;
                if (col >= g.N) continue;
                const floatx16_t &acv = acc[i][j];
                const float v[4] = {acv[4 * q], acv[4 * q + 1], acv[4 * q + 2], acv[4 * q + 3]};
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
                            const float4 zq = *reinterpret_cast<const float4 *>(zp);
                            zin[0] = zq.x; zin[1] = zq.y; zin[2] = zq.z; zin[3] = zq.w;
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

// BM x BN output tile per 256-thread workgroup; 2 x 2 waves, each with a
// (BM/2) x (BN/2) tile of TM x TN MFMA tiles of 32 x 32.  Runtime K loop,
// unrolled by the ring depth.
template <int BM, int BN, int BK, bool AK, bool BKc, int EPI, bool VEC>
__global__ void __launch_bounds__(NTHREADS, 2) gemm_bf16_kernel(GemmArgs g) {
    constexpr int PD = 2;   // K slabs in flight in registers ahead of the one multiplied
    group_offsets(g);
    if (gridDim.y > 1) {   // split K: this slice's rows of both operands, its own partial C
        const long long z = blockIdx.y;
        g.A += z * g.K * (AK ? 1 : g.lda);
        g.B += z * g.K * (BKc ? 1 : g.ldb);
        g.Cf += z * g.split_stride;
    }
    constexpr int TM = BM / 64, TN = BN / 64, LDS_LD = lds_ld<BK>();
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

    const int tid = threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);

    floatx16_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    // Global -> LDS pipeline: slab kt is in LDS buffer kt & 1 while the next
    // PD slabs are in flight in a ring of register sets.  Each step computes
    // from LDS, stores slab kt+1 into the other buffer and reuses its
    // registers for the load of slab kt+PD+1, so a load has PD steps of MFMA
    // work to arrive.  The ring index is a compile-time constant (the K loop
    // is unrolled by PD).
    constexpr int QA = BM * BK / 8 / NTHREADS, QB = BN * BK / 8 / NTHREADS;
    uint4 ra[PD][QA], rb[PD][QB];
    const int KT = (g.K + BK - 1) / BK;
    const __amdgpu_buffer_rsrc_t rsA =
        operand_rsrc(g.A, 2ll * g.lda * (AK ? g.M : g.K));
    const __amdgpu_buffer_rsrc_t rsB =
        operand_rsrc(g.B, 2ll * g.ldb * (BKc ? g.N : g.K));
    auto load_slab = [&](uint4 (&a)[QA], uint4 (&b)[QB], int kt) {
        load_tile<BM, BK, AK, VEC>(rsA, g.A, g.lda, m0, g.M, kt * BK, g.K, a, tid);
        load_tile<BN, BK, BKc, VEC>(rsB, g.B, g.ldb, n0, g.N, kt * BK, g.K, b, tid);
    };
    load_slab(ra[0], rb[0], 0);
    store_tile<BM, BK, AK>(sA[0], ra[0], tid);
    store_tile<BN, BK, BKc>(sB[0], rb[0], tid);
    __syncthreads();

    const int fr = lane & 31, fk = (lane >> 5) * 8;
    // MFMA fragments of one half slab (32 k = two MFMA k-steps of 16): a lane
    // holds 8 consecutive k of row (lane & 31) of each 32-row tile
    auto read_frags = [&](int cur, int kh, bf16x8_t (&af)[2][TM], bf16x8_t (&bfr)[2][TN]) {
        const uint16_t *A_ = sA[cur];
        const uint16_t *B_ = sB[cur];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
                af[s][i] = *reinterpret_cast<const bf16x8_t *>(A_ + (wm + i * 32 + fr) * LDS_LD + kh + 16 * s + fk);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                bfr[s][j] = *reinterpret_cast<const bf16x8_t *>(B_ + (wn + j * 32 + fr) * LDS_LD + kh + 16 * s + fk);
        }
    };
    auto mfma_frags = [&](const bf16x8_t (&af)[2][TM], const bf16x8_t (&bfr)[2][TN]) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = mfma32(bfr[s][j], af[s][i], acc[i][j]);
    };
    auto compute = [&](int cur) {
#pragma unroll
        for (int kh = 0; kh < BK; kh += 32) {
            bf16x8_t af[2][TM], bfr[2][TN];
            read_frags(cur, kh, af, bfr);
            mfma_frags(af, bfr);
        }
    };
    // one step: compute slab kt, store slab kt+1 (ring slot N) into the other
    // LDS buffer, then reuse slot N for the load of slab kt+PD+1
#define GEMM_STEP(KTV, N)                                                                 \
    compute((KTV) & 1);                                                                   \
    store_tile<BM, BK, AK>(sA[((KTV) + 1) & 1], ra[N], tid);                                   \
    store_tile<BN, BK, BKc>(sB[((KTV) + 1) & 1], rb[N], tid);                                  \
    lds_barrier();                                                                        \
    load_slab(ra[N], rb[N], (KTV) + PD + 1);
    if (KT == 1) {
        compute(0);
    } else {
        // KT rounded up to whole ring turns; the extra slabs load as zeros
        const int KTR = (KT + PD - 1) / PD * PD;
#pragma unroll
        for (int q = 1; q <= PD; ++q) load_slab(ra[q % PD], rb[q % PD], q);
        auto turn = [&](int kt) {
            GEMM_STEP(kt, 1)
            GEMM_STEP(kt + 1, 0)
        };
#pragma unroll 1
        for (int kt = 0; kt < KTR; kt += PD) turn(kt);
    }
#undef GEMM_STEP

    // the A operand buffers become the waves' output staging areas
    static_assert(2 * BM * LDS_LD >= 4 * (BM / 2) * (BN / 2 + 8), "staging fits in sA");
    __syncthreads();
    epilogue<BM, BN, EPI>(g, acc, m0, n0, wm, wn, lane, &sA[0][0] + wave * (BM / 2) * (BN / 2 + 8));
}

// Forward GEMM with the K slabs loaded straight into LDS (buffer loads with
// an LDS destination: no register staging, no LDS store instructions), for
// K-contiguous operands in whole 16-byte chunks and a compile-time slab
// count.  The LDS tiles are unpadded (128-byte rows); a lane's 16 bytes land
// at the wave's base + 16 lane, so the chunk order within a row is swizzled
// instead: LDS chunk position p of row r holds the operand's chunk
// p ^ ((r >> 1) & 7), which keeps the fragment reads of 16 consecutive rows
// on 16 distinct 4-bank groups.  Two stages, each its own LDS array (so the
// compiler can tell a load into one stage from reads of the other): slab
// kt+2 is loaded into the stage slab kt occupied once every wave has read it.
// The waits and barriers of the K loop are written out: the compiler's own
// fence would wait for every load into LDS, including the newest slab's.
template <int EPI, int KTC, int STAGES>
__global__ void __launch_bounds__(NTHREADS, 2) gemm_dma_kernel(GemmArgs g) {
    constexpr int BM = 128, BN = 128, BK = 64, TM = BM / 64, TN = BN / 64;
    constexpr int SA = BM * BK, SB = BN * BK;          // elements per operand and stage
    constexpr int NI = (BM + BN) * BK / 8 / NTHREADS;  // 16-byte loads per thread per slab
    static_assert(NI == 8, "the K loop waits for vmcnt(8)");
    constexpr int STG = (BM / 2) * (BN / 2 + 8);       // one wave's output staging area
    static_assert(SA >= STG && SB >= STG, "staging fits");
    // One LDS stage: operands and the four staging areas share one array
    // (37 KB), so that four workgroups fit on a CU and one's slab load and
    // barriers overlap the others' MFMAs (the kernel is latency-bound: with
    // two workgroups per CU its MFMA pipes are busy 40 % of the time and
    // its LDS 24 %).  Two stages (64 KB, two workgroups per CU): each
    // workgroup loads slab kt + 2 while it multiplies slab kt + 1; each
    // operand and stage then has its own array, so that the compiler sees
    // that the LDS-destination loads of one stage do not touch the other.
    static_assert(STAGES == 1 || (STAGES == 2 && KTC >= 2), "stages");
    constexpr bool ONE = STAGES == 1;
    constexpr int S1 = SA + SB > 4 * STG ? SA + SB : 4 * STG;
    __shared__ __attribute__((aligned(16))) uint16_t sA0[ONE ? S1 : SA], sB0[ONE ? 8 : SB],
        sA1[ONE ? 8 : SA], sB1[ONE ? 8 : SB];
    group_offsets(g);

    const int mt = (g.M + BM - 1) / BM, nt = (g.N + BN - 1) / BN;
    const int tiles = mt * nt;
    const int per = (tiles + 7) / 8;
    const int w = blockIdx.x;
    const int tile = (w & 7) * per + (w >> 3);
    if (tile >= tiles) return;
    const int tm = tile / nt, tn = tile - tm * nt;
    const int m0 = tm * BM, n0 = tn * BN;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);

    floatx16_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const __amdgpu_buffer_rsrc_t rsA = operand_rsrc(g.A, 2ll * g.lda * g.M);
    const __amdgpu_buffer_rsrc_t rsB = operand_rsrc(g.B, 2ll * g.ldb * g.N);
    // one slab: wave w loads rows [8 (4 w + q), +8) of A and of B, q < 4;
    // lane l: row 8 (4 w + q) + l / 8, LDS chunk l % 8, operand chunk swizzled
    auto load_slab = [&](int kt, uint16_t *sa, uint16_t *sb) {
        const int rl = lane >> 3, p = lane & 7, k0 = kt * BK;
#pragma unroll
        for (int q = 0; q < BM / 32; ++q) {
            const int r = (wave * (BM / 32) + q) * 8 + rl;
            const int gk = k0 + 8 * (p ^ ((r >> 1) & 7));
            const int offa = (m0 + r < g.M && gk < g.K) ? 2 * ((m0 + r) * g.lda + gk) : 0x7fffffff;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rsA, (void __attribute__((address_space(3))) *)(sa + (r - rl) * BK), 16, offa, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < BN / 32; ++q) {
            const int r = (wave * (BN / 32) + q) * 8 + rl;
            const int gk = k0 + 8 * (p ^ ((r >> 1) & 7));
            const int offb = (n0 + r < g.N && gk < g.K) ? 2 * ((n0 + r) * g.ldb + gk) : 0x7fffffff;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rsB, (void __attribute__((address_space(3))) *)(sb + (r - rl) * BK), 16, offb, 0, 0, 0);
        }
    };
    const int fr = lane & 31, fc = lane >> 5;   // fragment row in the tile, chunk within a k-step
    auto compute = [&](const uint16_t *sa, const uint16_t *sb) {
#pragma unroll
        for (int s = 0; s < BK / 16; ++s) {
            const int c = 2 * s + fc;   // logical 16-byte chunk of the row
            bf16x8_t af[TM], bfr[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int r = wm + i * 32 + fr;
                af[i] = *reinterpret_cast<const bf16x8_t *>(sa + r * BK + 8 * (c ^ ((r >> 1) & 7)));
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int r = wn + j * 32 + fr;
                bfr[j] = *reinterpret_cast<const bf16x8_t *>(sb + r * BK + 8 * (c ^ ((r >> 1) & 7)));
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = mfma32(bfr[j], af[i], acc[i][j]);
        }
    };
    if constexpr (ONE) {
#pragma unroll
        for (int kt = 0; kt < KTC; ++kt) {
            load_slab(kt, sA0, sA0 + SA);
            asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
            compute(sA0, sA0 + SA);
            // every wave has read the stage: it takes the next slab (or the output)
            asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        }
        epilogue<BM, BN, EPI>(g, acc, m0, n0, wm, wn, lane, sA0 + wave * STG);
    } else {
        load_slab(0, sA0, sB0);
        load_slab(1, sA1, sB1);
        asm volatile("s_waitcnt vmcnt(8)\n\ts_barrier" ::: "memory");
#pragma unroll
        for (int kt = 0; kt < KTC; ++kt) {
            uint16_t *sa = (kt & 1) ? sA1 : sA0, *sb = (kt & 1) ? sB1 : sB0;
            compute(sa, sb);
            if (kt + 1 < KTC) {
                // every wave has read this stage: it takes slab kt+2
                asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
                if (kt + 2 < KTC) {
                    load_slab(kt + 2, sa, sb);
                    asm volatile("s_waitcnt vmcnt(8)\n\ts_barrier" ::: "memory");   // slab kt+1 landed everywhere
                } else {
                    asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
                }
            }
        }
        // the stages become the waves' output staging areas, one array each
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        uint16_t *stage = wave == 0 ? sA0 : wave == 1 ? sB0 : wave == 2 ? sA1 : sB1;
        epilogue<BM, BN, EPI>(g, acc, m0, n0, wm, wn, lane, stage);
    }
}

#ifndef SPECIES_STAGES
#define SPECIES_STAGES 1   // LDS stages of the 25- and 13-slab instances
#endif

template <bool AKV, bool BKV, int EP>
static hipError_t launch_case(const GemmArgs &g, bool vec, hipStream_t s, int groups) {
    constexpr int TB = 128, TK = 64;
    const int tiles = ((g.M + TB - 1) / TB) * ((g.N + TB - 1) / TB);
    const dim3 grid(((tiles + 7) / 8) * 8, 1, groups);
    const int kt = (g.K + TK - 1) / TK;
    // forward layers of the MLP get a K loop unrolled for their slab count
    constexpr bool fwd =
        AKV && BKV && (EP == EPI_BIAS_GELU || EP == EPI_BIAS || EP == EPI_GELU_DOT || EP == EPI_GELU_GRAD);
#define GEMM_LAUNCH(VECV)                                                                    \
    hipLaunchKernelGGL((gemm_bf16_kernel<TB, TB, TK, AKV, BKV, EP, VECV>), dim3(grid),         \
                       dim3(NTHREADS), 0, s, g)
    if (!vec) {
        GEMM_LAUNCH(false);
    } else if constexpr (fwd) {
        // forward layers with a slab count the MLP has: slabs loaded straight into LDS
        // stages as measured fastest: one (four workgroups per CU) for 1, 8,
        // 13, 16 and 25 slabs; two for 4 slabs (the last layer, N = 32)
        if (kt == 1) hipLaunchKernelGGL((gemm_dma_kernel<EP, 1, 1>), dim3(grid), dim3(NTHREADS), 0, s, g);
        else if (kt == 16) hipLaunchKernelGGL((gemm_dma_kernel<EP, 16, 1>), dim3(grid), dim3(NTHREADS), 0, s, g);
        else if (kt == 8) hipLaunchKernelGGL((gemm_dma_kernel<EP, 8, 1>), dim3(grid), dim3(NTHREADS), 0, s, g);
        else if (kt == 4) hipLaunchKernelGGL((gemm_dma_kernel<EP, 4, 2>), dim3(grid), dim3(NTHREADS), 0, s, g);
        // the hidden layers of the per-species networks (1600 -> 800 -> 400,
        // K = 1600 and 832): 1.24 and 1.34 times faster than the register ring
        else if (kt == 25) hipLaunchKernelGGL((gemm_dma_kernel<EP, 25, SPECIES_STAGES>), dim3(grid), dim3(NTHREADS), 0, s, g);
        else if (kt == 13) hipLaunchKernelGGL((gemm_dma_kernel<EP, 13, SPECIES_STAGES>), dim3(grid), dim3(NTHREADS), 0, s, g);
        else GEMM_LAUNCH(true);
    } else {
        GEMM_LAUNCH(true);
    }
#undef GEMM_LAUNCH
    return hipGetLastError();
}

// C[i] = sum_z work[z][i], z in slice order (deterministic)
__global__ void splitk_reduce_kernel(const float *__restrict__ work, int split, long long count, float *C) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x) {
        float acc = 0.f;
#pragma unroll 8
        for (int z = 0; z < split; ++z) acc += work[z * count + i];
        C[i] = acc;
    }
}

hipError_t launch_gemm_splitk(const GemmArgs &g0, int split, float *work, hipStream_t s) {
    if (g0.M <= 0 || g0.N <= 0) return hipSuccess;
    if (split < 1 || g0.K % split != 0 || g0.ldc != g0.N) return hipErrorInvalidValue;
    if (split == 1) return launch_gemm(g0, false, false, EPI_STORE_F32, s);
    GemmArgs g = g0;
    g.K = g0.K / split;
    g.Cf = work;
    g.split_stride = (long long)g.M * g.N;
    const int64_t bytesA = 2ll * g.lda * g0.K, bytesB = 2ll * g.ldb * g0.K;
    if (bytesA >= (1ll << 31) || bytesB >= (1ll << 31)) return hipErrorInvalidValue;
    const bool vec = g.lda % 8 == 0 && g.M % 8 == 0 && g.ldb % 8 == 0 && g.N % 8 == 0;
    constexpr int TB = 128, TK = 64;
    const int tiles = ((g.M + TB - 1) / TB) * ((g.N + TB - 1) / TB);
    const dim3 grid(((tiles + 7) / 8) * 8, split);
    if (vec) hipLaunchKernelGGL((gemm_bf16_kernel<TB, TB, TK, false, false, EPI_STORE_F32, true>), grid,
                                dim3(NTHREADS), 0, s, g);
    else hipLaunchKernelGGL((gemm_bf16_kernel<TB, TB, TK, false, false, EPI_STORE_F32, false>), grid,
                            dim3(NTHREADS), 0, s, g);
    const long long count = (long long)g.M * g.N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)std::min<long long>(2048, (count + 255) / 256)),
                       dim3(256), 0, s, work, split, count, g0.Cf);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs &g, bool a_kcont, bool b_kcont, int epi, hipStream_t s, int groups) {
    if (g.M <= 0 || g.N <= 0 || groups == 0) return hipSuccess;
    if (g.K <= 0 || groups < 0 || groups > 65535) return hipErrorInvalidValue;
    // grouped operands must keep the alignment of the first group
    if (groups > 1 && (g.gsA % 8 != 0 || g.gsB % 8 != 0 || g.gsC % 8 != 0)) return hipErrorInvalidValue;
    // byte offsets of the buffer loads are 31-bit
    const int64_t bytesA = 2ll * g.lda * (a_kcont ? g.M : g.K);
    const int64_t bytesB = 2ll * g.ldb * (b_kcont ? g.N : g.K);
    if (bytesA >= (1ll << 31) || bytesB >= (1ll << 31)) return hipErrorInvalidValue;
    // whole 16-byte chunks in both operands: leading dimensions and chunked
    // extents multiples of 8 (then the branch-free buffer-load path)
    const bool vec = g.lda % 8 == 0 && (a_kcont ? g.K : g.M) % 8 == 0 && g.ldb % 8 == 0 &&
                     (b_kcont ? g.K : g.N) % 8 == 0;
    if (a_kcont && b_kcont) {
        switch (epi) {
            case EPI_BIAS_GELU: return launch_case<true, true, EPI_BIAS_GELU>(g, vec, s, groups);
            case EPI_BIAS: return launch_case<true, true, EPI_BIAS>(g, vec, s, groups);
            case EPI_GELU_GRAD: return launch_case<true, true, EPI_GELU_GRAD>(g, vec, s, groups);
            case EPI_STORE_F32: return launch_case<true, true, EPI_STORE_F32>(g, vec, s, groups);
            case EPI_GELU_DOT:
                // float4 reads of bias and weights; whole column quads
                if (!g.bias || !g.Zin || !g.Cf || g.N % 4 != 0 || ((uintptr_t)g.bias & 15) ||
                    ((uintptr_t)g.Zin & 15) || (groups > 1 && g.gsC % 4 != 0))
                    return hipErrorInvalidValue;
                return launch_case<true, true, EPI_GELU_DOT>(g, vec, s, groups);
            default: return hipErrorInvalidValue;
        }
    }
    if (!a_kcont && !b_kcont && epi == EPI_STORE_F32)
        return launch_case<false, false, EPI_STORE_F32>(g, vec, s, groups);
    return hipErrorInvalidValue;
}

}  // namespace chemk
