// chemk_dev.h -- device-side data layout and wave-level building blocks shared
// by the gfx950 kernels.
//
// One wavefront (64 lanes) owns one cell: lane k < K holds species k, lane K
// holds the temperature (y = (Y_1..Y_K, T), N = K + 1 <= 64).  Rates use cgs
// units inside (mol/cm^3, g/cm^3), which makes dY_k/dt = W_k omega_k / rho
// with W in g/mol.  Each wave has its own slice of LDS (see Lds); kernels that
// use these helpers launch one wave per workgroup or give every wave its own
// slice, and only synchronise inside the wave.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chemk {

constexpr int WAVE = 64;
constexpr double RU_CGS = 8.31446261815324e7;        // erg/(mol K)
constexpr double RU_SI = 8.31446261815324;           // J/(mol K)
constexpr double RC_CAL = 8.31446261815324 / 4.184;  // cal/(mol K)
constexpr double P0_CGS = 101325.0 * 10.0;           // standard pressure, dyn/cm^2
constexpr double PA_TO_CGS = 10.0;                   // Pa -> dyn/cm^2
constexpr double LN_P0_RU = -4.407418589020958141;   // ln(P0_CGS / RU_CGS)

// Mechanism tables in device memory.
struct DevMech {
    int K, R, E, N;          // N = K + 1
    const double *W;         // [K] g/mol
    const double *invW;      // [K]
    const double *nasa;      // [K*7]
    const int4 *rsp;         // [R] reactant slots 0/1, product slots 0/1 (-1 empty)
    const double4 *rpar;     // [R] (ln A, beta, Ea/R_c [K], 0)
    const int4 *rflag;       // [R] (third body, reversible, dnu, n_f + 16 n_r)
    const int *inc_start;    // [K+1] CSR over species of the reactions touching k
    const int *inc_r;        // [nnz]
    const double *inc_nu;    // [nnz] net stoichiometric coefficient of k in r
    const double *Emat;      // [E*K] mass fraction of element e carried by species k
};

// ---------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// The lane index as an opaque value: per-lane table addresses derived from it
// are recomputed where they are used instead of being hoisted out of the
// integration loop as long-lived 64-bit register pairs (cheap to rebuild,
// expensive to keep: they push the DI kernel into scratch spills).
__device__ __forceinline__ int lane_fresh() {
    int l = threadIdx.x & (WAVE - 1);
    asm volatile("" : "+v"(l));
    return l;
}

// Orders LDS traffic of this wave around the call (compiler and memory model).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// wave-uniform copy of a double (the value of the first active lane)
__device__ __forceinline__ double uniform_d(double v) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// DPP lane exchanges inside a row of 16 lanes: a VALU operand modifier, so no
// LDS round trip (ds_bpermute) per step.  quad_perm [1,0,3,2] and [2,3,0,1]
// swap neighbours at distance 1 and 2, the mirrors pair the two quads of a
// half row and the two half rows of a row.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <int CTRL> __device__ __forceinline__ unsigned dpp_u(unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

template <int CTRL> __device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// value of v in lane src (src wave-uniform)
__device__ __forceinline__ double bcast(double v, int src) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// Sum over the wave as one wave-uniform value: four DPP steps leave every
// lane with its 16-lane row sum, the four row sums are read as scalars and
// added in a fixed order.  Uniform by construction (the per-lane partial
// sums may differ in the last bit: the compiler can fuse a lane's own
// product into the first step, and branches must never see such values).
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<kDppXor1>(v);
    v += dpp_d<kDppXor2>(v);
    v += dpp_d<kDppHalfMirror>(v);
    v += dpp_d<kDppMirror>(v);
    return (bcast(v, 0) + bcast(v, 16)) + (bcast(v, 32) + bcast(v, 48));
}

// Pivot search: the lane of (about) the largest v >= 0 among lanes with cand
// set, wave-uniform.  The 32-bit key holds a candidate bit, the exponent and
// the top 14 mantissa bits of v (non-negative doubles order like unsigned
// integers) and the lane in the 6 low bits: candidates within a relative 6e-5
// of each other are tie-broken to the lowest lane (partial pivoting needs a
// large pivot, not the largest to the last bit: |l| <= 1 + 6e-5).  One DPP
// max per step, then the four row maxima as scalars.
__device__ __forceinline__ int wave_argmax(double v, bool cand) {
    const int lane = lane_id();
    const unsigned hi = (unsigned)__double2hiint(v);
    unsigned key = cand ? (0x80000000u | (hi & 0x7fffffc0u) | (unsigned)(63 - lane)) : 0u;
    key = max(key, dpp_u<kDppXor1>(key));
    key = max(key, dpp_u<kDppXor2>(key));
    key = max(key, dpp_u<kDppHalfMirror>(key));
    key = max(key, dpp_u<kDppMirror>(key));
    const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)key, 0);
    const unsigned r1 = (unsigned)__builtin_amdgcn_readlane((int)key, 16);
    const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)key, 32);
    const unsigned r3 = (unsigned)__builtin_amdgcn_readlane((int)key, 48);
    const unsigned best = max(max(r0, r1), max(r2, r3));
    return 63 - (int)(best & 63u);
}

// ---------------------------------------------------------------------------
// NASA-7 of one species
// ---------------------------------------------------------------------------
struct SpThermo {
    double cpR, hRT, sR, dcpR;   // cp/R, h/RT, s/R, d(cp/R)/dT
};

__device__ __forceinline__ SpThermo sp_thermo(const double *a, double T, double lnT,
                                              double invT) {
    SpThermo t;
    const double T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    t.cpR = a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4;
    t.hRT = a[0] + a[1] * T * 0.5 + a[2] * T2 * (1.0 / 3.0) + a[3] * T3 * 0.25 +
            a[4] * T4 * 0.2 + a[5] * invT;
    t.sR = a[0] * lnT + a[1] * T + a[2] * T2 * 0.5 + a[3] * T3 * (1.0 / 3.0) +
           a[4] * T4 * 0.25 + a[6];
    t.dcpR = a[1] + 2.0 * a[2] * T + 3.0 * a[3] * T2 + 4.0 * a[4] * T3;
    return t;
}

__device__ __forceinline__ void sp_cp_h(const double *a, double T, double invT, double &cpR,
                                        double &hRT) {
    const double T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    cpR = a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4;
    hRT = a[0] + a[1] * T * 0.5 + a[2] * T2 * (1.0 / 3.0) + a[3] * T3 * 0.25 + a[4] * T4 * 0.2 +
          a[5] * invT;
}

// ---------------------------------------------------------------------------
// per-wave LDS slice
// ---------------------------------------------------------------------------
struct Lds {
    double *C, *gRT, *hRT, *cpR;   // [64] each
    double *u, *tcol, *hs;         // [64] Jacobian assembly vectors
    double *w;                     // [64] net production rates (accumulated per reaction)
    int *piv;                      // [64]
    double *J;                     // [ld * ld] Jacobian rows, leading dimension ld
    int ld;
};

__host__ __device__ inline int lds_doubles_per_wave(int K, int R, int ld) {
    return 8 * 64 + 32 + ld * ld;
}

// The matrix comes first, so that a row's columns sit within the short
// immediate offsets of the LDS instructions from the row's address.
__device__ __forceinline__ Lds carve_lds(double *base, int K, int R, int ld) {
    Lds L;
    L.J = base;
    double *v = base + ld * ld;
    L.C = v;
    L.gRT = v + 64;
    L.hRT = v + 128;
    L.cpR = v + 192;
    L.u = v + 256;
    L.tcol = v + 320;
    L.hs = v + 384;
    L.w = v + 448;
    L.piv = reinterpret_cast<int *>(v + 512);
    L.ld = ld;
    return L;
}

// Natural logarithm of x > 0 (NaN for x <= 0 and for NaN): x = 2^e m with
// m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s), s = (m - 1) / (m + 1),
// |s| <= 0.1716, by its Taylor series to s^21 (the first omitted term is
// below 2e-19 of the sum), and e ln 2 with ln 2 split in two parts (Cody and
// Waite) so that e ln2_hi is exact.  About a third of the instructions of the
// library's log, within 2 ulp of the exact value.
__device__ __forceinline__ double ln_pos(double x) {
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752440) {
        m = m + m;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 1.0 / 21.0;
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    const double de = (double)e;
    const double lo = fma(de, 1.9082149292705877000e-10, 2.0 * (s * z * p));
    const double r = fma(de, 6.9314718036912381649e-01, lo + 2.0 * s);
    return x > 0.0 ? r : __builtin_nan("");
}

// Per-cell scalars that the Jacobian and the right-hand side share.
struct CellScalars {
    double T, invT, lnT, Wbar, rho, M;
};

__device__ __forceinline__ CellScalars cell_scalars(const DevMech &m, double p_cgs, double y,
                                                    double Yk, double iw) {
    CellScalars c;
    c.T = bcast(y, m.K);
    c.invT = 1.0 / c.T;
    c.lnT = ln_pos(c.T);
    c.Wbar = 1.0 / wave_sum(Yk * iw);
    c.rho = p_cgs * c.Wbar * c.invT / RU_CGS;   // g/cm^3
    c.M = p_cgs * c.invT / RU_CGS;              // mol/cm^3
    return c;
}

// Rate constants and fluxes of reaction r (the law of the header comment).
struct RxnEval {
    double lnkf, qf, qr, dlnKc_T, dHr;   // dlnKc_T = d ln Kc / dT, dHr = sum nu h/RT
    double kfM, krM;                     // k_f [M] and k_r [M] ([M] = 1 without third body)
};

__device__ __forceinline__ RxnEval rxn_eval(const DevMech &m, const Lds &L, int r,
                                            const CellScalars &c, double lnPref, int4 s4,
                                            double4 pr, int4 fl, bool want_T) {
    RxnEval e;
    e.lnkf = pr.x + pr.y * c.lnT - pr.z * c.invT;
    const double kf = exp(e.lnkf);
    const double Ma = fl.x ? c.M : 1.0;
    e.kfM = kf * Ma;
    e.krM = 0.0;
    e.qf = e.kfM * L.C[s4.x] * (s4.y >= 0 ? L.C[s4.y] : 1.0);
    e.qr = 0.0;
    e.dlnKc_T = 0.0;
    e.dHr = 0.0;
    if (fl.y) {
        const double dg = L.gRT[s4.z] + (s4.w >= 0 ? L.gRT[s4.w] : 0.0) - L.gRT[s4.x] -
                          (s4.y >= 0 ? L.gRT[s4.y] : 0.0);
        const double lnKc = -dg + fl.z * lnPref;
        e.krM = exp(e.lnkf - lnKc) * Ma;
        e.qr = e.krM * L.C[s4.z] * (s4.w >= 0 ? L.C[s4.w] : 1.0);
        if (want_T) {
            e.dHr = L.hRT[s4.z] + (s4.w >= 0 ? L.hRT[s4.w] : 0.0) - L.hRT[s4.x] -
                    (s4.y >= 0 ? L.hRT[s4.y] : 0.0);
            e.dlnKc_T = (e.dHr - fl.z) * c.invT;
        }
    } else if (want_T) {
        e.dHr = (s4.z >= 0 ? L.hRT[s4.z] : 0.0) + (s4.w >= 0 ? L.hRT[s4.w] : 0.0) -
                L.hRT[s4.x] - (s4.y >= 0 ? L.hRT[s4.y] : 0.0);
    }
    return e;
}

// Wave-cooperative right-hand side: f for this lane's component (0 on lanes
// >= N).  Lane k < K holds Y_k in y, lane K holds T.
__device__ __forceinline__ double wave_rhs(const DevMech &m, const Lds &L, double p_cgs,
                                           double y) {
    const int lane = lane_fresh();
    const int K = m.K;
    const bool sp = lane < K;
    const double Yk = sp ? y : 0.0;
    const double iw = sp ? m.invW[lane] : 0.0;
    const CellScalars c = cell_scalars(m, p_cgs, y, Yk, iw);
    double cpR = 0.0, hRT = 0.0;
    if (sp) {
        SpThermo t = sp_thermo(m.nasa + 7 * lane, c.T, c.lnT, c.invT);
        cpR = t.cpR;
        hRT = t.hRT;
        L.C[lane] = c.rho * Yk * iw;
        L.gRT[lane] = t.hRT - t.sR;
    }
    L.w[lane] = 0.0;
    wave_sync();
    const double lnPref = LN_P0_RU - c.lnT;   // ln(p0 / (R T))
    // each reaction adds its net rate to its participants' production rates
    // (LDS atomics in a fixed lane and loop order)
#pragma unroll 1
    for (int r = lane; r < m.R; r += WAVE) {
        const int4 s4 = m.rsp[r];
        RxnEval e = rxn_eval(m, L, r, c, lnPref, s4, m.rpar[r], m.rflag[r], false);
        const double q = e.qf - e.qr;
        atomicAdd(&L.w[s4.x], -q);
        if (s4.y >= 0) atomicAdd(&L.w[s4.y], -q);
        if (s4.z >= 0) atomicAdd(&L.w[s4.z], q);
        if (s4.w >= 0) atomicAdd(&L.w[s4.w], q);
    }
    wave_sync();
    const double wk = sp ? L.w[lane] : 0.0;
    const double chat = wave_sum(Yk * cpR * iw);     // sum_k Y_k (cp_k/R) / W_k
    const double Q = wave_sum(hRT * wk);             // sum_k (h_k/RT) omega_k
    wave_sync();
    if (sp) return m.W[lane] * wk / c.rho;
    if (lane == K) return -c.T * Q / (c.rho * chat);
    return 0.0;
}

// Wave-cooperative f and analytic Jacobian at y.  Rows of J go to L.J (row i
// = component i, leading dimension L.ld); returns this lane's f.
//
// With C_i = rho Y_i/W_i, rho = p Wbar/(R T) and S_kj = sum_r nu_kr dq_r/dC_j:
//   J_kj = (W_k/W_j) S_kj + (Wbar/W_j) (f_k - W_k u_k / rho),  u_k = sum_i S_ki C_i
//   J_kT = (W_k/rho) (tcol_k - u_k/T) + f_k / T,  tcol_k = sum_r nu_kr dq_r/dT|_C
// and for f_T = -T Q/(rho chat), Q = sum_k (h_k/RT) omega_k:
//   J_Tj = (1/W_j) [ -(T/chat) hs_j + (T Wbar/(rho chat)) Hu - f_T (cp_j/R - chat Wbar)/chat ]
//   J_TT = -2Q/(rho chat) - T Q'/(rho chat) + T Q chat'/(rho chat^2)
// with hs_j = sum_r dH_r dq_r/dC_j, Hu = sum_k (h_k/RT) u_k, Q' = dQ/dT, chat' = dchat/dT.
__device__ __forceinline__ double wave_f_jac(const DevMech &m, const Lds &L, double p_cgs,
                                             double y) {
    const int lane = lane_fresh();
    const int K = m.K, ld = L.ld;
    const bool sp = lane < K;
    const double Yk = sp ? y : 0.0;
    const double iw = sp ? m.invW[lane] : 0.0;
    const CellScalars c = cell_scalars(m, p_cgs, y, Yk, iw);
    SpThermo t = {0.0, 0.0, 0.0, 0.0};
    if (sp) {
        t = sp_thermo(m.nasa + 7 * lane, c.T, c.lnT, c.invT);
        L.C[lane] = c.rho * Yk * iw;
        L.gRT[lane] = t.hRT - t.sR;
        L.hRT[lane] = t.hRT;
        L.cpR[lane] = t.cpR;
        L.u[lane] = 0.0;
        L.tcol[lane] = 0.0;
        L.hs[lane] = 0.0;
        L.w[lane] = 0.0;
#pragma unroll 1
        for (int j = 0; j < K; ++j) L.J[lane * ld + j] = 0.0;
    }
    wave_sync();
    const double lnPref = LN_P0_RU - c.lnT;   // ln(p0 / (R T))
#pragma unroll 1
    for (int r = lane; r < m.R; r += WAVE) {
        const int4 s4 = m.rsp[r];
        const double4 pr = m.rpar[r];
        const int4 fl = m.rflag[r];
        RxnEval e = rxn_eval(m, L, r, c, lnPref, s4, pr, fl, true);
        const double q = e.qf - e.qr;
        atomicAdd(&L.w[s4.x], -q);
        if (s4.y >= 0) atomicAdd(&L.w[s4.y], -q);
        if (s4.z >= 0) atomicAdd(&L.w[s4.z], q);
        if (s4.w >= 0) atomicAdd(&L.w[s4.w], q);
        const double dlnkf = (pr.y + pr.z * c.invT) * c.invT;
        const double dlnM = fl.x ? -c.invT : 0.0;
        const double dqdT = e.qf * (dlnkf + dlnM) - e.qr * (dlnkf - e.dlnKc_T + dlnM);
        const int nf = fl.w & 15, nr = fl.w >> 4;
        const double D = nf * e.qf - nr * e.qr;        // sum_i C_i dq/dC_i
        // participants: slot species and stoichiometric sign
        const int sp_[4] = {s4.x, s4.y, s4.z, s4.w};
        const double nu_[4] = {-1.0, -1.0, 1.0, 1.0};
        // dq/dC of each slot (product rule, so a doubled species gets both terms)
        double dq_[4];
        dq_[0] = e.kfM * (s4.y >= 0 ? L.C[s4.y] : 1.0);
        dq_[1] = s4.y >= 0 ? e.kfM * L.C[s4.x] : 0.0;
        dq_[2] = -e.krM * (s4.w >= 0 ? L.C[s4.w] : 1.0);
        dq_[3] = s4.w >= 0 ? -e.krM * L.C[s4.z] : 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int k = sp_[a];
            if (k < 0) continue;
            atomicAdd(&L.u[k], nu_[a] * D);
            atomicAdd(&L.tcol[k], nu_[a] * dqdT);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = sp_[b];
                if (j < 0 || dq_[b] == 0.0) continue;
                atomicAdd(&L.J[k * ld + j], nu_[a] * dq_[b]);
            }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int j = sp_[b];
            if (j < 0 || dq_[b] == 0.0) continue;
            atomicAdd(&L.hs[j], e.dHr * dq_[b]);
        }
    }
    wave_sync();
    const double wk = sp ? L.w[lane] : 0.0;
    const double uk = sp ? L.u[lane] : 0.0;
    const double tk = sp ? L.tcol[lane] : 0.0;
    const double chat = wave_sum(Yk * t.cpR * iw);
    const double Q = wave_sum(t.hRT * wk);
    const double Hu = wave_sum(t.hRT * uk);
    const double Qp = wave_sum((t.cpR - t.hRT) * c.invT * wk + t.hRT * (tk - uk * c.invT));
    const double chatp = wave_sum(Yk * t.dcpR * iw);
    const double fT = -c.T * Q / (c.rho * chat);
    double f = 0.0;
    if (sp) {
        const double Wk = m.W[lane];
        f = Wk * wk / c.rho;
        const double rank1 = c.Wbar * (f - Wk * uk / c.rho);
        for (int j = 0; j < K; ++j) {
            const double ij = m.invW[j];
            L.J[lane * ld + j] = Wk * ij * L.J[lane * ld + j] + ij * rank1;
        }
        L.J[lane * ld + K] = (Wk / c.rho) * (tk - uk * c.invT) + f * c.invT;
    } else if (lane == K) {
        f = fT;
        const double ichat = 1.0 / chat;
        const double a1 = -c.T * ichat;
        const double a2 = c.T * c.Wbar * Hu / (c.rho * chat);
        const double a3 = fT * ichat;
        for (int j = 0; j < K; ++j) {
            const double ij = m.invW[j];
            L.J[K * ld + j] = ij * (a1 * L.hs[j] + a2 - a3 * (L.cpR[j] - chat * c.Wbar));
        }
        L.J[K * ld + K] = -2.0 * Q / (c.rho * chat) - c.T * Qp / (c.rho * chat) +
                          c.T * Q * chatp / (c.rho * chat * chat);
    }
    wave_sync();
    return f;
}

}  // namespace chemk
