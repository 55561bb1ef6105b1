// props.hip -- property kernels on gfx950: mixture cp and h, T from h (Newton),
// and the RHS / Jacobian evaluation hooks.
//
// The property update of the method (Sec. II.A) evaluates temperature
// polynomials and inverts h(T) by Newton's method per cell.  These kernels are
// HBM-bound streams: a 64-lane workgroup copies a contiguous block of 64 rows
// of Y (64*K doubles, coalesced) into LDS, then each lane works on one cell
// from LDS (row stride K+1 to spread the banks).
#include "chemk_dev.h"
#include "chemk_internal.h"

namespace chemk {

constexpr int PROP_CELLS = 64;

__device__ __forceinline__ int64_t stage_rows(const double *__restrict__ Y, int64_t base,
                                              int64_t n, int K, double *sY) {
    const int64_t cnt64 = n - base < PROP_CELLS ? n - base : PROP_CELLS;
    const int cnt = (int)cnt64;
    const double *src = Y + base * K;
    const int ld = K + 1;
    for (int i = threadIdx.x; i < cnt * K; i += blockDim.x) {
        const int c = i / K, k = i - c * K;
        sY[c * ld + k] = src[i];
    }
    __syncthreads();
    return cnt;
}

// mixture cp/R and h/(RT), per unit mass (mol/g), for one cell row in LDS
__device__ __forceinline__ void mix_cp_h(const DevMech &m, const double *y, double T,
                                         double &cR, double &hRT) {
    const double invT = 1.0 / T;
    double c = 0.0, h = 0.0;
    for (int k = 0; k < m.K; ++k) {
        double cpR, hk;
        sp_cp_h(m.nasa + 7 * k, T, invT, cpR, hk);
        const double yw = y[k] * m.invW[k];
        c += yw * cpR;
        h += yw * hk;
    }
    cR = c;
    hRT = h;
}

__global__ void __launch_bounds__(PROP_CELLS) thermo_kernel(DevMech m, int64_t n,
                                                            const double *__restrict__ T,
                                                            const double *__restrict__ Y,
                                                            double *cp, double *h) {
    extern __shared__ double sY[];
    const int ld = m.K + 1;
    for (int64_t base = (int64_t)blockIdx.x * PROP_CELLS; base < n;
         base += (int64_t)gridDim.x * PROP_CELLS) {
        const int cnt = (int)stage_rows(Y, base, n, m.K, sY);
        if ((int)threadIdx.x < cnt) {
            const int64_t c = base + threadIdx.x;
            const double Tc = T[c];
            double cR, hRT;
            mix_cp_h(m, sY + threadIdx.x * ld, Tc, cR, hRT);
            cp[c] = cR * RU_SI * 1e3;          // J/(kg K)
            h[c] = hRT * Tc * RU_SI * 1e3;     // J/kg
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(PROP_CELLS) T_from_h_kernel(DevMech m, int64_t n,
                                                              const double *__restrict__ hin,
                                                              const double *__restrict__ Y,
                                                              double *T, int *status) {
    extern __shared__ double sY[];
    const int ld = m.K + 1;
    for (int64_t base = (int64_t)blockIdx.x * PROP_CELLS; base < n;
         base += (int64_t)gridDim.x * PROP_CELLS) {
        const int cnt = (int)stage_rows(Y, base, n, m.K, sY);
        if ((int)threadIdx.x < cnt) {
            const int64_t c = base + threadIdx.x;
            const double *y = sY + threadIdx.x * ld;
            const double h0R = hin[c] / (RU_SI * 1e3);   // h/R per gram
            double Tg = T[c];
            int st = 1;   // 1 = not converged yet
            for (int it = 0; it < 50; ++it) {
                double cR, hRT;
                mix_cp_h(m, y, Tg, cR, hRT);
                const double dT = (hRT * Tg - h0R) / cR;
                Tg -= dT;
                if (!isfinite(Tg)) break;
                if (fabs(dT) <= 1e-12 * fabs(Tg)) {
                    if (Tg >= 200.0 && Tg <= 4000.0) st = 0;
                    break;
                }
            }
            if (st) {
                double lo = 200.0, hi = 4000.0, cR, hlo, hhi;
                mix_cp_h(m, y, lo, cR, hlo);
                mix_cp_h(m, y, hi, cR, hhi);
                hlo *= lo;
                hhi *= hi;
                if (hlo <= h0R && h0R <= hhi) {
                    for (int it = 0; it < 200 && hi - lo > 1e-13 * hi; ++it) {
                        const double mid = 0.5 * (lo + hi);
                        double hm;
                        mix_cp_h(m, y, mid, cR, hm);
                        if (hm * mid < h0R) lo = mid;
                        else hi = mid;
                    }
                    Tg = 0.5 * (lo + hi);
                    st = 0;
                } else {
                    st = CHEMK_CELL_NEWTON;
                }
            }
            if (st == 0) T[c] = Tg;
            status[c] = st;
        }
        __syncthreads();
    }
}

// one wave per cell: f (and J) through the same device functions as DI
__global__ void __launch_bounds__(64) rhs_kernel(DevMech m, int64_t n, const double *T,
                                                 const double *p, const double *Y,
                                                 double *dydt) {
    extern __shared__ double lds[];
    const Lds L = carve_lds(lds, m.K, m.R, 1);
    const int lane = lane_id();
    const int K = m.K, N = K + 1;
    for (int64_t c = blockIdx.x; c < n; c += gridDim.x) {
        double y = 0.0;
        if (lane < K) y = Y[c * K + lane];
        else if (lane == K) y = T[c];
        const double f = wave_rhs(m, L, p[c] * PA_TO_CGS, y);
        if (lane < N) dydt[c * N + lane] = f;
    }
}

__global__ void __launch_bounds__(64) jacobian_kernel(DevMech m, int ld, int64_t n,
                                                      const double *T, const double *p,
                                                      const double *Y, double *J) {
    extern __shared__ double lds[];
    const Lds L = carve_lds(lds, m.K, m.R, ld);
    const int lane = lane_id();
    const int K = m.K, N = K + 1;
    for (int64_t c = blockIdx.x; c < n; c += gridDim.x) {
        double y = 0.0;
        if (lane < K) y = Y[c * K + lane];
        else if (lane == K) y = T[c];
        (void)wave_f_jac(m, L, p[c] * PA_TO_CGS, y);
        double *out = J + c * N * N;
        for (int i = lane; i < N * N; i += WAVE) {
            const int r = i / N, col = i - r * N;
            out[i] = L.J[r * ld + col];
        }
        wave_sync();
    }
}

static int grid_for(int64_t n, int64_t cap) { return (int)(n < cap ? n : cap); }

hipError_t launch_thermo(const DevMech &m, int64_t n, const double *T, const double *Y,
                         double *cp, double *h, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * PROP_CELLS * (m.K + 1);
    hipLaunchKernelGGL(thermo_kernel, dim3(grid_for((n + PROP_CELLS - 1) / PROP_CELLS, 8192)),
                       dim3(PROP_CELLS), lds, s, m, n, T, Y, cp, h);
    return hipGetLastError();
}

hipError_t launch_T_from_h(const DevMech &m, int64_t n, const double *h, const double *Y,
                           double *T, int *status, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * PROP_CELLS * (m.K + 1);
    hipLaunchKernelGGL(T_from_h_kernel, dim3(grid_for((n + PROP_CELLS - 1) / PROP_CELLS, 8192)),
                       dim3(PROP_CELLS), lds, s, m, n, h, Y, T, status);
    return hipGetLastError();
}

hipError_t launch_rhs(const DevMech &m, int64_t n, const double *T, const double *p,
                      const double *Y, double *dydt, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const size_t lds = di_lds_bytes(m.K, m.R, 1);
    hipLaunchKernelGGL(rhs_kernel, dim3(grid_for(n, 16384)), dim3(64), lds, s, m, n, T, p, Y,
                       dydt);
    return hipGetLastError();
}

hipError_t launch_jacobian(const DevMech &m, int64_t n, const double *T, const double *p,
                           const double *Y, double *J, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int ld = m.K + 1;
    const size_t lds = di_lds_bytes(m.K, m.R, ld);
    hipLaunchKernelGGL(jacobian_kernel, dim3(grid_for(n, 16384)), dim3(64), lds, s, m, ld, n, T,
                       p, Y, J);
    return hipGetLastError();
}

}  // namespace chemk
