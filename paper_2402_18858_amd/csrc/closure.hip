// closure.hip -- the steps on either side of the chemistry advance on gfx950:
// the transport-property update (Sec. II.A: properties from temperature
// polynomials) and the PaSR closure that consumes the advance's output
// (Sec. III: chemical time from the slowest species formation rate, mixing
// time the geometric mean of the sub-grid and Kolmogorov times).  Lane k
// of a cell's lanes works on species k: two cells per wavefront for
// mechanisms of at most 32 species, one per wavefront above that.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "chemk.h"
#include "chemk_dev.h"
#include "chemk_internal.h"

using namespace chemk;

void ctx_set_error(const char *msg);
chemk::DevMech ctx_devmech(chemk_ctx *c);
int ctx_device(chemk_ctx *c);
void *&ctx_transport(chemk_ctx *c);

namespace {

// Device tables of the transport model: ln(mu_k) and ln(lambda_k) as cubic
// polynomials in ln T [K*4 each], and Wilke's factors w_ij = (W_j/W_i)^(1/4),
// c_ij = (8 (1 + W_i/W_j))^(-1/2) [K*K each].
struct Transport {
    double *d = nullptr;   // one allocation: mu [4K], lam [4K], w [K K], c [K K]
    int K = 0;
};

constexpr double R_SI = 8.31446261815324;

// max over the wave (every lane gets it)
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

__device__ __forceinline__ double poly3_exp(const double *c, double lt) {
    return exp(c[0] + lt * (c[1] + lt * (c[2] + lt * c[3])));
}

// One wave per cell: mixture viscosity (Wilke) and conductivity (Mathur,
// Tondon and Saxena) from the species polynomials, the factor table read
// from global memory (mechanisms whose table does not fit a workgroup's LDS).
__global__ void __launch_bounds__(256) transport_kernel(DevMech m, const double *__restrict__ tab, int n,
                                                        const double *__restrict__ T, const double *__restrict__ Y,
                                                        double *mu_out, double *lam_out) {
    const int K = m.K;
    const int lane = lane_id();
    // the wave's cell, as a scalar: whole waves leave together
    const int c = uniform((int)(blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE)));
    if (c >= n) return;
    const bool sp = lane < K;
    const double *muc = tab, *lac = tab + 4 * K, *wt = tab + 8 * K, *ct = wt + K * K;
    const double Tc = T[c];
    const double lt = ln_pos(Tc);
    const double Yk = sp ? Y[(size_t)c * K + lane] : 0.0;
    const double nk = sp ? Yk * m.invW[lane] : 0.0;
    const double X = nk / wave_sum(nk);
    const double mu = sp ? poly3_exp(muc + 4 * lane, lt) : 1.0;
    const double lam = sp ? poly3_exp(lac + 4 * lane, lt) : 1.0;
    const double s = sqrt(mu);
    double den = 0.0;
    for (int j = 0; j < K; ++j) {
        const double Xj = bcast(X, j), sj = bcast(s, j);
        if (sp) {
            const double f = 1.0 + (s / sj) * wt[lane * K + j];
            den += Xj * f * f * ct[lane * K + j];
        }
    }
    const double mix = wave_sum(sp ? X * mu / den : 0.0);
    const double la = wave_sum(sp ? X * lam : 0.0);
    const double lh = wave_sum(sp ? X / lam : 0.0);
    if (lane == 0) {
        mu_out[c] = mix;
        if (lam_out) lam_out[c] = 0.5 * (la + 1.0 / lh);
    }
}

// Mechanisms of at most 32 species: two cells per wave, lanes 32 h + i on
// species i of the wave's cell h.  Sums and maxima stay within a half.
constexpr int HALF = 32;

__device__ __forceinline__ double half_sum(double v) {
#pragma unroll
    for (int o = HALF / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ double half_max(double v) {
#pragma unroll
    for (int o = HALF / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

constexpr int PAIR_WAVES = 4;                  // waves per workgroup

// Sum over the LN = WAVE / CPW lanes of one cell (CPW cells per wave).
template <int CPW> __device__ __forceinline__ double cell_sum(double v) {
#pragma unroll
    for (int o = WAVE / CPW / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Transport, CPW cells per wave (2 for K <= 32, else 1), lane i of a cell's
// lanes on species i.  Each workgroup stages Wilke's factors once in LDS
// (dynamic, K K pairs (w_ij, c_ij) at j K + i, so that a cell's lanes read
// consecutive pairs for each j) and then walks the cells PAIR_WAVES CPW at
// a time.  Each lane keeps sqrt(mu_i) and publishes its reciprocal, with
// its mole fraction, in LDS for the cell's j loop.
template <int CPW>
__global__ void __launch_bounds__(64 * PAIR_WAVES) transport_lds_kernel(DevMech m, const double *__restrict__ tab,
                                                                        int n, const double *__restrict__ T,
                                                                        const double *__restrict__ Y, double *mu_out,
                                                                        double *lam_out) {
    constexpr int LN = WAVE / CPW;   // lanes per cell
    constexpr int CELLS = PAIR_WAVES * CPW;
    extern __shared__ double2 wc[];   // [K K]
    __shared__ double2 xs[PAIR_WAVES][CPW][LN];
    const int K = m.K;
    const double *muc = tab, *lac = tab + 4 * K, *wt = tab + 8 * K, *ct = wt + K * K;
    for (int t = threadIdx.x; t < K * K; t += blockDim.x) {
        const int j = t / K, i = t - j * K;
        wc[t] = make_double2(wt[i * K + j], ct[i * K + j]);
    }
    const int lane = lane_id();
    const int h = lane / LN, i = lane % LN;
    const int w = threadIdx.x / WAVE;
    const bool sp = i < K;
    const int ii = sp ? i : 0;   // lanes past K read a valid pair, unused
    for (int base = blockIdx.x * CELLS; base < n; base += gridDim.x * CELLS) {
        __syncthreads();   // the table is in place; the last pass's xs is read
        const int c = base + CPW * w + h;
        const bool live = c < n;
        const double Tc = live ? T[c] : 1000.0;
        const double lt = ln_pos(Tc);
        const double nk = (sp && live) ? Y[(size_t)c * K + i] * m.invW[i] : 0.0;
        const double tot = cell_sum<CPW>(nk);
        const double X = live ? nk / tot : 0.0;
        const double mu = sp ? poly3_exp(muc + 4 * i, lt) : 1.0;
        const double lam = sp ? poly3_exp(lac + 4 * i, lt) : 1.0;
        const double s = sqrt(mu);
        xs[w][h][i] = make_double2(X, 1.0 / s);
        __syncthreads();
        double den = 0.0;
        for (int j = 0; j < K; ++j) {
            const double2 xj = xs[w][h][j];
            const double2 p = wc[j * K + ii];
            const double f = fma(s * xj.y, p.x, 1.0);
            den = fma(f * f, xj.x * p.y, den);
        }
        const double mix = cell_sum<CPW>(sp ? X * mu / den : 0.0);
        const double la = cell_sum<CPW>(sp ? X * lam : 0.0);
        const double lh = cell_sum<CPW>(sp ? X / lam : 0.0);
        if (i == 0 && live) {
            mu_out[c] = mix;
            if (lam_out) lam_out[c] = 0.5 * (la + 1.0 / lh);
        }
    }
}

constexpr int PASR_PAIRS = 4;   // cell pairs per wave

// The PaSR closure (see pasr_kernel) of K <= 32 species, two cells per wave
// and PASR_PAIRS pairs per wave, adjacent in memory: every load of the
// wave's cells is issued before the first pair's arithmetic, so that more
// bytes are in flight per wave.
__global__ void __launch_bounds__(256) pasr_pair_kernel(DevMech m, int n, const double *__restrict__ T,
                                                        const double *__restrict__ p, const double *__restrict__ Y0,
                                                        const double *__restrict__ Y1, double dt,
                                                        const double *__restrict__ ksgs,
                                                        const double *__restrict__ delta,
                                                        const double *__restrict__ mu, double c_eps, double y_min,
                                                        double *kappa_out, double *omega_out, double *Yout) {
    const int K = m.K;
    const int lane = lane_id();
    const int h = lane / HALF, i = lane % HALF;
    const int wave = (int)(blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE);
    const double invW = i < K ? m.invW[i] : 0.0;
    double y0[PASR_PAIRS], y1[PASR_PAIRS], Tc[PASR_PAIRS], pc[PASR_PAIRS], kc[PASR_PAIRS], dc[PASR_PAIRS],
        mc[PASR_PAIRS];
#pragma unroll
    for (int q = 0; q < PASR_PAIRS; ++q) {
        const int c = (wave * PASR_PAIRS + q) * 2 + h;
        const bool live = c < n;
        const bool sp = live && i < K;
        y0[q] = sp ? Y0[(size_t)c * K + i] : 0.0;
        y1[q] = sp ? Y1[(size_t)c * K + i] : 0.0;
        Tc[q] = live ? T[c] : 1.0;
        pc[q] = live ? p[c] : 1.0;
        kc[q] = live ? ksgs[c] : 0.0;
        dc[q] = live ? delta[c] : 1.0;
        mc[q] = live ? mu[c] : 1.0;
    }
#pragma unroll
    for (int q = 0; q < PASR_PAIRS; ++q) {
        const int c = (wave * PASR_PAIRS + q) * 2 + h;
        const bool live = c < n;
        const bool sp = live && i < K;
        const double rho = pc[q] / (R_SI * Tc[q] * half_sum(sp ? y0[q] * invW * 1e3 : 0.0));
        const double om = rho * (y1[q] - y0[q]) / dt;
        const double tk = (sp && om > 0.0 && y1[q] >= y_min) ? rho * y1[q] / om : -1.0;
        const double tau_c = half_max(tk);
        double kappa = 1.0;
        if (tau_c >= 0.0) {
            const double k = kc[q];
            if (k <= 0.0) {
                kappa = 0.0;
            } else {
                const double up = sqrt(2.0 * k / 3.0);
                const double tau_d = dc[q] / up;
                const double eps = c_eps * k * sqrt(k) / dc[q];
                const double tau_k = sqrt(mc[q] / rho / eps);
                const double tau_mix = sqrt(tau_d * tau_k);
                kappa = tau_c / (tau_c + tau_mix);
            }
        }
        if (sp) {
            if (omega_out) omega_out[(size_t)c * K + i] = kappa * om;
            if (Yout) Yout[(size_t)c * K + i] = y0[q] + kappa * (y1[q] - y0[q]);
        }
        if (live && i == 0 && kappa_out) kappa_out[c] = kappa;
    }
}

// One wave per cell: the PaSR closure of one step (see chemk_pasr).
__global__ void __launch_bounds__(256) pasr_kernel(DevMech m, int n, const double *__restrict__ T,
                                                   const double *__restrict__ p, const double *__restrict__ Y0,
                                                   const double *__restrict__ Y1, double dt,
                                                   const double *__restrict__ ksgs, const double *__restrict__ delta,
                                                   const double *__restrict__ mu, double c_eps, double y_min,
                                                   double *kappa_out, double *omega_out, double *Yout) {
    const int K = m.K;
    const int lane = lane_id();
    const int c = uniform((int)(blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE)));
    if (c >= n) return;
    const bool sp = lane < K;
    const double y0 = sp ? Y0[(size_t)c * K + lane] : 0.0;
    const double y1 = sp ? Y1[(size_t)c * K + lane] : 0.0;
    // density of the step's initial state [kg/m^3]
    const double rho = p[c] / (R_SI * T[c] * wave_sum(sp ? y0 * m.invW[lane] * 1e3 : 0.0));
    const double om = rho * (y1 - y0) / dt;
    const double tk = (sp && om > 0.0 && y1 >= y_min) ? rho * y1 / om : -1.0;
    const double tau_c = wave_max(tk);
    double kappa = 1.0;
    if (tau_c >= 0.0) {
        const double k = ksgs[c];
        if (k <= 0.0) {
            kappa = 0.0;
        } else {
            const double up = sqrt(2.0 * k / 3.0);
            const double tau_d = delta[c] / up;
            const double eps = c_eps * k * sqrt(k) / delta[c];
            const double tau_k = sqrt(mu[c] / rho / eps);
            const double tau_mix = sqrt(tau_d * tau_k);
            kappa = tau_c / (tau_c + tau_mix);
        }
    }
    if (sp) {
        if (omega_out) omega_out[(size_t)c * K + lane] = kappa * om;
        if (Yout) Yout[(size_t)c * K + lane] = y0 + kappa * (y1 - y0);
    }
    if (lane == 0 && kappa_out) kappa_out[c] = kappa;
}

int fail_arg(const char *msg) {
    ctx_set_error(msg);
    return CHEMK_E_ARG;
}

}  // namespace

namespace chemk {
void transport_destroy(void *t) {
    Transport *tr = static_cast<Transport *>(t);
    if (!tr) return;
    (void)hipFree(tr->d);
    delete tr;
}
}  // namespace chemk

extern "C" int chemk_transport_set(chemk_ctx *c, const double *mu_poly, const double *lam_poly) {
    ctx_set_error("");
    if (!c || !mu_poly || !lam_poly) return fail_arg("null argument");
    const DevMech m = ctx_devmech(c);
    const int K = m.K;
    for (int i = 0; i < 4 * K; ++i)
        if (!std::isfinite(mu_poly[i]) || !std::isfinite(lam_poly[i])) return fail_arg("non-finite coefficient");
    // molar masses from the device tables' host copy: read them back once
    std::vector<double> W(K);
    if (hipSetDevice(ctx_device(c)) != hipSuccess ||
        hipMemcpy(W.data(), m.W, 8 * (size_t)K, hipMemcpyDeviceToHost) != hipSuccess) {
        ctx_set_error("reading the molar masses");
        return CHEMK_E_HIP;
    }
    std::vector<double> h(8 * (size_t)K + 2 * (size_t)K * K);
    std::memcpy(h.data(), mu_poly, 32 * (size_t)K);
    std::memcpy(h.data() + 4 * K, lam_poly, 32 * (size_t)K);
    double *w = h.data() + 8 * K, *cf = w + (size_t)K * K;
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j) {
            w[i * K + j] = std::pow(W[j] / W[i], 0.25);
            cf[i * K + j] = 1.0 / std::sqrt(8.0 * (1.0 + W[i] / W[j]));
        }
    void *&slot = ctx_transport(c);
    Transport *tr = static_cast<Transport *>(slot);
    if (!tr) {
        tr = new Transport;
        slot = tr;
    }
    if (tr->K != K || !tr->d) {
        (void)hipFree(tr->d);
        tr->d = nullptr;
        if (hipMalloc(&tr->d, 8 * h.size()) != hipSuccess) {
            ctx_set_error("transport tables");
            return CHEMK_E_OOM;
        }
        tr->K = K;
    }
    if (hipMemcpy(tr->d, h.data(), 8 * h.size(), hipMemcpyHostToDevice) != hipSuccess) {
        ctx_set_error("transport tables upload");
        return CHEMK_E_HIP;
    }
    return CHEMK_OK;
}

extern "C" int chemk_transport(chemk_ctx *c, int64_t n, const double *T, const double *Y, double *mu,
                               double *lam, void *stream) {
    ctx_set_error("");
    if (!c) return fail_arg("null context");
    Transport *tr = static_cast<Transport *>(ctx_transport(c));
    if (!tr || !tr->d) {
        ctx_set_error("transport coefficients not set (chemk_transport_set)");
        return CHEMK_E_STATE;
    }
    if (n < 0 || n > (1ll << 31) - 1) return fail_arg("bad n");
    if (n == 0) return CHEMK_OK;
    if (!T || !Y || !mu) return fail_arg("null array");
    if (hipSetDevice(ctx_device(c)) != hipSuccess) return CHEMK_E_HIP;
    // about eight workgroups per CU, each staging the factor table once
    const size_t lds = sizeof(double2) * (size_t)tr->K * tr->K;
    if (tr->K <= HALF) {
        const int64_t passes = (n + 2 * PAIR_WAVES - 1) / (2 * PAIR_WAVES);
        hipLaunchKernelGGL(transport_lds_kernel<2>, dim3((unsigned)std::min<int64_t>(passes, 2048)),
                           dim3(64 * PAIR_WAVES), lds, (hipStream_t)stream, ctx_devmech(c), tr->d, (int)n, T, Y, mu,
                           lam);
    } else if (lds + sizeof(double2) * WAVE * PAIR_WAVES <= 64 * 1024) {
        const int64_t passes = (n + PAIR_WAVES - 1) / PAIR_WAVES;
        hipLaunchKernelGGL(transport_lds_kernel<1>, dim3((unsigned)std::min<int64_t>(passes, 2048)),
                           dim3(64 * PAIR_WAVES), lds, (hipStream_t)stream, ctx_devmech(c), tr->d, (int)n, T, Y, mu,
                           lam);
    } else {
        const int per = 4;   // cells (waves) per workgroup
        hipLaunchKernelGGL(transport_kernel, dim3((unsigned)((n + per - 1) / per)), dim3(64 * per), 0,
                           (hipStream_t)stream, ctx_devmech(c), tr->d, (int)n, T, Y, mu, lam);
    }
    if (hipGetLastError() != hipSuccess) {
        ctx_set_error("transport launch");
        return CHEMK_E_HIP;
    }
    return CHEMK_OK;
}

extern "C" int chemk_pasr(chemk_ctx *c, int64_t n, const double *T, const double *p, const double *Y0,
                          const double *Y1, double dt, const double *k_sgs, const double *delta, const double *mu,
                          double c_eps, double y_min, double *kappa, double *omega, double *Y_out, void *stream) {
    ctx_set_error("");
    if (!c) return fail_arg("null context");
    if (n < 0 || n > (1ll << 31) - 1) return fail_arg("bad n");
    if (n == 0) return CHEMK_OK;
    if (!T || !p || !Y0 || !Y1 || !k_sgs || !delta || !mu) return fail_arg("null array");
    if (!kappa && !omega && !Y_out) return fail_arg("no output requested");
    if (!(dt > 0) || !std::isfinite(dt)) return fail_arg("dt must be finite and > 0");
    if (!(c_eps > 0) || !std::isfinite(c_eps) || !(y_min >= 0) || !std::isfinite(y_min))
        return fail_arg("c_eps must be > 0 and y_min >= 0");
    if (hipSetDevice(ctx_device(c)) != hipSuccess) return CHEMK_E_HIP;
    const DevMech dm = ctx_devmech(c);
    if (dm.K <= HALF) {
        const int64_t per = 4 * 2 * PASR_PAIRS;   // cells per workgroup of four waves
        hipLaunchKernelGGL(pasr_pair_kernel, dim3((unsigned)((n + per - 1) / per)), dim3(256), 0,
                           (hipStream_t)stream, dm, (int)n, T, p, Y0, Y1, dt, k_sgs, delta, mu, c_eps, y_min, kappa,
                           omega, Y_out);
    } else {
        const int per = 4;
        hipLaunchKernelGGL(pasr_kernel, dim3((unsigned)((n + per - 1) / per)), dim3(64 * per), 0,
                           (hipStream_t)stream, dm, (int)n, T, p, Y0, Y1, dt, k_sgs, delta, mu, c_eps, y_min, kappa,
                           omega, Y_out);
    }
    if (hipGetLastError() != hipSuccess) {
        ctx_set_error("PaSR launch");
        return CHEMK_E_HIP;
    }
    return CHEMK_OK;
}
