// di.hip -- direct integration (DI) of the per-cell kinetics ODEs (Eq. 1) over one
// flow step (Eq. 2) on gfx950.
//
// Design: one wavefront per cell.  Lane i < N holds component i of
// y = (Y_1..Y_K, T) and owns row i of the Jacobian / iteration matrix
// (1/(h gamma)) I - J in the wave's LDS slice.  LU with partial pivoting reads
// each pivot row from LDS and keeps the permutation implicit; the triangular
// solves gather the right-hand side in pivot order and broadcast one solution
// component per step.  All loop control is wave-uniform by construction.
// Integrator: RODAS (Hairer & Wanner, Solving ODEs II, Sec. VI.4), the
// stiffly accurate Rosenbrock method of order 4 with an embedded order-3
// estimate, in its transformed form; weighted-RMS error control.
// Scheduling: a persistent grid pulls cells from a queue with one atomic per
// cell; the queue is ordered by a stiffness estimate (expensive bins first)
// so that the tail of the launch is short.
#include "chemk_dev.h"
#include "chemk_internal.h"

namespace chemk {

// RODAS coefficients, transformed form (published values, Hairer & Wanner).
__constant__ double kA[6][5] = {
    {0, 0, 0, 0, 0},
    {1.544, 0, 0, 0, 0},
    {0.9466785280815826, 0.2557011698983284, 0, 0, 0},
    {3.314825187068521, 2.896124015972201, 0.9986419139977817, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0}};
__constant__ double kC[6][5] = {
    {0, 0, 0, 0, 0},
    {-5.6688, 0, 0, 0, 0},
    {-2.430093356833875, -0.2063599157091915, 0, 0, 0},
    {-0.1073529058151375, -9.594562251023355, -20.47028614809616, 0, 0},
    {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.70890893206160, 0},
    {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136,
     -6.058818238834054}};
constexpr double kGamma = 0.25;

// ---------------------------------------------------------------------------
// dense LU of the iteration matrix in LDS, one row per lane, implicit
// partial pivoting (the pivot row is read from LDS by every lane; rows are not
// moved).
// On return: L.piv[k] = row chosen at step k; that row holds its L
// multipliers in columns < k and U in columns >= k; mystep = the step at
// which this lane's row was chosen.  Returns false on an exactly zero pivot.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool wave_lu(const Lds &L, int n, int &mystep) {
    const int lane = lane_id();
    double *row = L.J + lane * L.ld;
    mystep = lane < n ? n : -1;
    bool ok = true;
    // ak: this lane's entry in the current pivot column, carried in a register
    // from one step to the next (the update of column k+1 is done first)
    double ak = lane < n ? row[0] : 0.0;
#pragma unroll 1
    for (int k = 0; k < n; ++k) {
        const bool open = mystep == n;
        const int p = wave_argmax(fabs(ak), open);
        const double pv = bcast(ak, p);   // the pivot, from the pivot lane's register
        if (lane == p) {
            mystep = k;
            L.piv[k] = p;
        }
        if (pv == 0.0) ok = false;
        const double *prow = L.J + p * L.ld;
        double next = 0.0;
        if (mystep == n) {   // rows still open (the pivot row itself is now closed)
            const double l = ak / pv;
            row[k] = l;
            int j = k + 1;
            if (j < n) {
                next = row[j] - l * prow[j];
                row[j] = next;
                ++j;
            }
            // four columns per pass: all eight LDS reads are issued before the
            // first use, so one wait covers them (the row update is otherwise a
            // chain of load latencies)
#pragma unroll 1
            for (; j + 4 <= n; j += 4) {
                const double p0 = prow[j], p1 = prow[j + 1], p2 = prow[j + 2], p3 = prow[j + 3];
                const double r0 = row[j], r1 = row[j + 1], r2 = row[j + 2], r3 = row[j + 3];
                row[j] = r0 - l * p0;
                row[j + 1] = r1 - l * p1;
                row[j + 2] = r2 - l * p2;
                row[j + 3] = r3 - l * p3;
            }
#pragma unroll 1
            for (; j < n; ++j) row[j] -= l * prow[j];
        }
        ak = next;
        wave_sync();
    }
    return ok;
}

// Solve (LU) x = b; b is this lane's component (equation `lane`), the
// solution component of variable i is returned in lane i.  Lane k works on
// the row chosen at step k (LDS row src = piv[k]); rdiag = 1/U_kk.
__device__ __forceinline__ double wave_solve(const Lds &L, int n, int src, double rdiag,
                                             double b) {
    const int lane = lane_id();
    const double *row = L.J + src * L.ld;
    // right-hand side in pivot order
    double z = __shfl(b, src, WAVE);
    // forward: L y = Pb (unit lower triangle).  The matrix entries of four
    // steps are read ahead (they do not depend on z); the broadcasts stay in
    // order.
    const bool in = lane < n;
    int k = 0;
#pragma unroll 1
    for (; k + 4 <= n - 1; k += 4) {
        const double a0 = row[k], a1 = row[k + 1], a2 = row[k + 2], a3 = row[k + 3];
        double zk = bcast(z, k);
        if (in && lane > k) z -= a0 * zk;
        zk = bcast(z, k + 1);
        if (in && lane > k + 1) z -= a1 * zk;
        zk = bcast(z, k + 2);
        if (in && lane > k + 2) z -= a2 * zk;
        zk = bcast(z, k + 3);
        if (in && lane > k + 3) z -= a3 * zk;
    }
#pragma unroll 1
    for (; k < n - 1; ++k) {
        const double zk = bcast(z, k);
        if (in && lane > k) z -= row[k] * zk;
    }
    // backward: U x = y
    k = n - 1;
#pragma unroll 1
    for (; k >= 3; k -= 4) {
        const double a0 = row[k], a1 = row[k - 1], a2 = row[k - 2], a3 = row[k - 3];
        double xk = bcast(z * rdiag, k);
        if (lane < k) z -= a0 * xk;
        if (lane == k) z = xk;
        xk = bcast(z * rdiag, k - 1);
        if (lane < k - 1) z -= a1 * xk;
        if (lane == k - 1) z = xk;
        xk = bcast(z * rdiag, k - 2);
        if (lane < k - 2) z -= a2 * xk;
        if (lane == k - 2) z = xk;
        xk = bcast(z * rdiag, k - 3);
        if (lane < k - 3) z -= a3 * xk;
        if (lane == k - 3) z = xk;
    }
#pragma unroll 1
    for (; k >= 0; --k) {
        const double xk = bcast(z * rdiag, k);
        if (lane < k) z -= row[k] * xk;
        if (lane == k) z = xk;
    }
    return in ? z : 0.0;
}

// ---------------------------------------------------------------------------
// Register-resident LU for a system of fixed size NT (instantiated for the
// sizes of the shipped mechanisms).  The rows stay in place (implicit partial
// pivoting, as above) but lane p keeps row p in NT registers: the loops over
// columns are unrolled, so every column index is a register index and the
// elimination reads only the pivot row from LDS (one broadcast read per two
// columns).  At step k every lane writes its columns right of k into its LDS
// row (one store per two columns for the whole wave, with no branch on the
// pivot lane), and the open rows read the pivot row from there.  (The
// compiler copies a row's registers before storing them, two moves per
// column; stores written in inline assembly avoided the copies but left the
// 54-column instance, whose registers spill to the accumulation registers,
// giving other numbers than the LDS LU, so the stores stay compiler-made.)  Afterwards
// each lane keeps its L multipliers (columns < its step) in registers and
// zeros elsewhere, and its LDS row holds U strictly right of the diagonal and
// zeros elsewhere, so the forward and backward sweeps need no lane masks.  The matrix factorised is
// A = J - fac I, the negated iteration matrix: the multipliers and pivots
// are exactly those of the LDS LU of fac I - J, with signs flipped where
// they enter, so both paths give the same numbers.
// ---------------------------------------------------------------------------
template <int NT>
struct RegLU {
    double a[NT];                 // L multipliers of this lane's row (columns < its step), else 0
    double rdiag;                 // 1 / U diagonal of this lane's row (lanes < NT)
    unsigned pkp[(NT + 4) / 5];   // lane of the row chosen at step k, 6 bits each, 5 per word
    int src;                      // lane of the row chosen at step `lane` (lanes < NT)
    // the pivot lane of step k (k a compile-time index: scalar shifts only)
    __device__ __forceinline__ int pk(int k) const { return (int)((pkp[k / 5] >> (6 * (k % 5))) & 63u); }
};

// Step K of the factorisation (and, recursively, the steps after it).
template <int K, int NT>
__device__ __forceinline__ void reg_lu_steps(const Lds &L, RegLU<NT> &f, double *row, bool in, int &mystep,
                                             bool &ok) {
    if constexpr (K < NT) {
        const int lane = lane_id();
        const int p = wave_argmax(fabs(f.a[K]), mystep == NT);
        f.pkp[K / 5] |= (unsigned)p << (6 * (K % 5));
        const double pv = bcast(f.a[K], p);
        if (pv == 0.0) ok = false;
        if (lane == p) {
            mystep = K;
            L.tcol[lane] = pv;   // the diagonal (L.tcol is free until the next Jacobian)
            L.piv[K] = lane;
        }
        // every row publishes its columns right of K (closed rows republish
        // what they already hold); the pivot row is read from there
        if (in) {
#pragma unroll
            for (int c = K + 1; c < NT; ++c) row[c] = f.a[c];
        }
        wave_sync();
        if (mystep == NT) {
            const double *prow = L.J + p * L.ld;
            const double l = f.a[K] / pv;
            f.a[K] = l;
#pragma unroll
            for (int c = K + 1; c < NT; ++c) f.a[c] = f.a[c] - l * prow[c];
        }
        reg_lu_steps<K + 1, NT>(L, f, row, in, mystep, ok);
    }
}

template <int NT>
__device__ __forceinline__ bool reg_lu(const Lds &L, double fac, RegLU<NT> &f) {
    const int lane = lane_id();
    const bool in = lane < NT;
    double *row = L.J + (in ? lane : 0) * L.ld;
    if (in) {
        row[lane] -= fac;
#pragma unroll
        for (int c = 0; c < NT; ++c) f.a[c] = row[c];
    } else {
#pragma unroll
        for (int c = 0; c < NT; ++c) f.a[c] = 0.0;
    }
    int mystep = in ? NT : -1;
    bool ok = true;
#pragma unroll
    for (int w = 0; w < (NT + 4) / 5; ++w) f.pkp[w] = 0u;
    reg_lu_steps<0, NT>(L, f, row, in, mystep, ok);
    // registers: L strictly left of the lane's step; LDS row: U strictly right
    if (in) {
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            row[c] = c > mystep ? f.a[c] : 0.0;
            if (c >= mystep) f.a[c] = 0.0;
        }
    }
    f.rdiag = in ? 1.0 / L.tcol[lane] : 0.0;
    f.src = in ? L.piv[lane] : 0;
    wave_sync();
    return ok;
}

// Solve (fac I - J) x = b with the factors of reg_lu; b is this lane's
// component, x_i is returned in lane i.
template <int NT>
__device__ __forceinline__ double reg_solve(const Lds &L, const RegLU<NT> &f, double b) {
    const int lane = lane_id();
    const bool in = lane < NT;
    double acc = in ? -b : 0.0;
    // forward (L y = P(-b)): lane p accumulates until its own step broadcasts it
#pragma unroll
    for (int k = 0; k < NT; ++k) acc = acc - f.a[k] * bcast(acc, f.pk(k));
    // backward (U x = y): U rows from LDS, zero left of and on the diagonal
    const double *row = L.J + (in ? lane : 0) * L.ld;
#pragma unroll
    for (int k = NT - 1; k >= 0; --k) acc = acc - row[k] * bcast(acc * f.rdiag, f.pk(k));
    const double x = acc * f.rdiag;   // the unknown of this lane's step
    const double r = __shfl(x, f.src, WAVE);
    return in ? r : 0.0;
}

struct DIParams {
    double rtol, atolY, atolT, h0_frac;
    int max_steps, project;
};

// Element projection of the lane's Y_k onto the element masses of Yin
// (weights w_k = max(Y_k, 1e-30)):  Y <- Y - w E^T (E w E^T)^-1 (E Y - E Yin).
// The E x E system is assembled with wave sums, solved by lane 0 in LDS
// (partial pivoting) and the multipliers are read back by every lane.
__device__ __forceinline__ double wave_project(const DevMech &m, const Lds &L, double Yk,
                                               double Yin) {
    const int lane = lane_id();
    const int K = m.K, E = m.E;
    const bool sp = lane < K;
    const double w = sp ? fmax(Yk, 1e-30) : 0.0;
    double *A = L.u;    // [E*E]
    double *r = L.hs;   // [E]
    for (int a = 0; a < E; ++a) {
        const double Ea = sp ? m.Emat[a * K + lane] : 0.0;
        const double ra = wave_sum(Ea * Yk) - wave_sum(Ea * Yin);
        if (lane == 0) r[a] = ra;
        for (int b = a; b < E; ++b) {
            const double Eb = sp ? m.Emat[b * K + lane] : 0.0;
            const double v = wave_sum(Ea * w * Eb);
            if (lane == 0) {
                A[a * E + b] = v;
                A[b * E + a] = v;
            }
        }
    }
    wave_sync();
    if (lane == 0) {
        bool ok = true;
        for (int k = 0; k < E && ok; ++k) {
            int p = k;
            double best = fabs(A[k * E + k]);
            for (int i = k + 1; i < E; ++i)
                if (fabs(A[i * E + k]) > best) {
                    best = fabs(A[i * E + k]);
                    p = i;
                }
            if (best == 0.0) {
                ok = false;
                break;
            }
            if (p != k) {
                for (int j = 0; j < E; ++j) {
                    const double t = A[k * E + j];
                    A[k * E + j] = A[p * E + j];
                    A[p * E + j] = t;
                }
                const double t = r[k];
                r[k] = r[p];
                r[p] = t;
            }
            for (int i = k + 1; i < E; ++i) {
                const double l = A[i * E + k] / A[k * E + k];
                for (int j = k; j < E; ++j) A[i * E + j] -= l * A[k * E + j];
                r[i] -= l * r[k];
            }
        }
        if (ok) {
            for (int i = E - 1; i >= 0; --i) {
                for (int j = i + 1; j < E; ++j) r[i] -= A[i * E + j] * r[j];
                r[i] /= A[i * E + i];
            }
        } else {
            for (int i = 0; i < E; ++i) r[i] = 0.0;
        }
    }
    wave_sync();
    double acc = 0.0;
    for (int e = 0; e < E; ++e) acc += (sp ? m.Emat[e * K + lane] : 0.0) * r[e];
    wave_sync();
    return sp ? Yk - w * acc : Yk;
}

// Mixture enthalpy h/R [K mol/g] and cp/R [mol/g] (per unit mass, R factored out).
__device__ __forceinline__ void wave_h_cp(const DevMech &m, double T, double Yk, double &hR,
                                          double &cR) {
    const int lane = lane_id();
    double cpR = 0.0, hRT = 0.0, iw = 0.0;
    const double invT = 1.0 / T;
    if (lane < m.K) {
        sp_cp_h(m.nasa + 7 * lane, T, invT, cpR, hRT);
        iw = m.invW[lane];
    }
    hR = wave_sum(Yk * hRT * iw) * T;
    cR = wave_sum(Yk * cpR * iw);
}

// Newton on h(T) = h0 then bisection on [200, 4000] K (same rule as the
// property kernel).  Returns 0 or CHEMK_CELL_NEWTON.
__device__ __forceinline__ int wave_T_from_h(const DevMech &m, double h0R, double Yk,
                                             double &T) {
    double Tg = T;
    for (int it = 0; it < 50; ++it) {
        double hR, cR;
        wave_h_cp(m, Tg, Yk, hR, cR);
        const double dT = (hR - h0R) / cR;
        Tg -= dT;
        if (!isfinite(Tg)) break;
        if (fabs(dT) <= 1e-12 * fabs(Tg)) {
            if (Tg >= 200.0 && Tg <= 4000.0) {
                T = Tg;
                return 0;
            }
            break;
        }
    }
    double lo = 200.0, hi = 4000.0, hlo, hhi, c;
    wave_h_cp(m, lo, Yk, hlo, c);
    wave_h_cp(m, hi, Yk, hhi, c);
    if (!(hlo <= h0R && h0R <= hhi)) return CHEMK_CELL_NEWTON;
    for (int it = 0; it < 200 && hi - lo > 1e-13 * hi; ++it) {
        const double mid = 0.5 * (lo + hi);
        double hm;
        wave_h_cp(m, mid, Yk, hm, c);
        if (hm < h0R) lo = mid;
        else hi = mid;
    }
    T = 0.5 * (lo + hi);
    return 0;
}

// Integrate one cell over dt.  y: this lane's component (in/out).  Returns the
// cell status; nsteps receives the number of attempted steps.  All loop
// control (t, h, error, counters) is wave-uniform by construction.
// NT > 0 factorises with the register-resident LU of size NT (= K + 1), NT = 0
// with the LDS LU of any size; both give the same numbers.  The six stages
// run as one loop (one copy of the right-hand side and of the solve in the
// code), the stage sums taken over all earlier stages with the published
// coefficients (zero past the stage's own).
template <int NT>
__device__ int di_cell(const DevMech &m, const Lds &L, double p_cgs, double &y, double dt,
                       const DIParams &o, int &nsteps) {
    const int lane = lane_id();
    const int K = m.K, Na = K + 1;
    const bool act = lane < Na;
    const double atol = lane < K ? o.atolY : o.atolT;
    const double yin = y;
    // conserved enthalpy at the start
    double h0R, cdummy;
    wave_h_cp(m, bcast(y, K), lane < K ? y : 0.0, h0R, cdummy);

    double f0 = 0.0;
    double t = 0.0, h = o.h0_frac * dt;
    bool rejected = false;
    int nst = 0, status = 0;
    int mystep = -1;
    RegLU<(NT > 0 ? NT : 1)> f;
#pragma unroll 1
    for (int guard = 0; guard <= o.max_steps; ++guard) {
        if (!(t < dt)) break;
        if (nst >= o.max_steps) {
            status = CHEMK_CELL_MAX_STEPS;
            break;
        }
        bool last = false;
        if (t + h >= dt * (1.0 - 1e-14) || t + h >= dt) {
            h = dt - t;
            last = true;
        }
        if (h <= 1e-20 * dt || h <= 0.0) {
            status = CHEMK_CELL_MAX_STEPS;
            break;
        }
        // the Jacobian at y (a rejected step re-evaluates it, as the method's
        // order conditions assume the exact J at the step's start)
        f0 = wave_f_jac(m, L, p_cgs, y);
        ++nst;
        const double fac = 1.0 / (h * kGamma);
        int src = 0;
        double rdiag = 0.0;
        if constexpr (NT > 0) {
            if (!reg_lu<NT>(L, fac, f)) {
                status = CHEMK_CELL_SINGULAR;
                break;
            }
        } else {
            // iteration matrix fac I - J in place of J
            if (act) {
                double *row = L.J + lane * L.ld;
                row[lane] = fac - row[lane];
#pragma unroll 1
                for (int j = 0; j < Na; ++j)
                    if (j != lane) row[j] = -row[j];
            }
            wave_sync();
            if (!wave_lu(L, Na, mystep)) {
                status = CHEMK_CELL_SINGULAR;
                break;
            }
            // lanes past the system read row 0 (in the slice; their results are unused)
            src = act ? L.piv[lane] : 0;
            rdiag = act ? 1.0 / L.J[src * L.ld + lane] : 0.0;
        }
        const double ih = 1.0 / h;
        double u0 = 0.0, u1 = 0.0, u2 = 0.0, u3 = 0.0, u4 = 0.0, u5 = 0.0;
        double yt = y;
#pragma unroll 1
        for (int s = 0; s < 6; ++s) {
            double rhs = f0;
            if (s > 0) {
                yt = y;
                yt += kA[s][0] * u0;
                yt += kA[s][1] * u1;
                yt += kA[s][2] * u2;
                yt += kA[s][3] * u3;
                yt += kA[s][4] * u4;
                const double fs = wave_rhs(m, L, p_cgs, yt);
                double cs = kC[s][0] * u0;
                cs += kC[s][1] * u1;
                cs += kC[s][2] * u2;
                cs += kC[s][3] * u3;
                cs += kC[s][4] * u4;
                rhs = fs + ih * cs;
            }
            double us;
            if constexpr (NT > 0) us = reg_solve<NT>(L, f, rhs);
            else us = wave_solve(L, Na, src, rdiag, rhs);
            switch (s) {
                case 0: u0 = us; break;
                case 1: u1 = us; break;
                case 2: u2 = us; break;
                case 3: u3 = us; break;
                case 4: u4 = us; break;
                default: u5 = us; break;
            }
        }
        const double ynew = yt + u5;   // yt: the embedded (order 3) solution of the last stage
        const double sc = atol + o.rtol * fmax(fabs(y), fabs(ynew));
        const double e = act ? u5 / sc : 0.0;
        const double err = uniform_d(sqrt(wave_sum(e * e) / Na));
        if (!isfinite(err)) {
            h = uniform_d(h * 0.2);
            rejected = true;
            continue;
        }
        if (err <= 1.0) {
            t = uniform_d(last ? dt : t + h);
            y = act ? ynew : 0.0;
            double fc = err > 0.0 ? 0.9 / sqrt(sqrt(err)) : 5.0;
            fc = fmin(5.0, fmax(0.2, fc));
            if (rejected) fc = fmin(fc, 1.0);
            h = uniform_d(h * fc);
            rejected = false;
        } else {
            h = uniform_d(h * fmax(0.2, 0.9 / sqrt(sqrt(err))));
            rejected = true;
        }
    }
    if (status == 0 && t < dt) status = CHEMK_CELL_MAX_STEPS;
    nsteps = nst;
    if (status == 0) {
        // non-finite state anywhere -> status 3
        const double bad = isfinite(y) ? 0.0 : 1.0;
        if (wave_sum(bad) > 0.0) status = CHEMK_CELL_NONFINITE;
    }
    if (status == 0) {
        double Yk = lane < K ? y : 0.0;
        if (o.project) Yk = wave_project(m, L, Yk, lane < K ? yin : 0.0);
        double T = bcast(y, K);
        const int st = wave_T_from_h(m, h0R, Yk, T);
        if (st) {
            status = st;
        } else {
            y = lane < K ? Yk : (lane == K ? T : 0.0);
            if (T < 200.0 || T > 4000.0) status = CHEMK_CELL_T_RANGE;
        }
    }
    if (status != 0 && status != CHEMK_CELL_T_RANGE) y = yin;   // leave the state untouched
    return status;
}

// Waves per workgroup of the DI kernel; each wave has its own LDS slice and
// its own cells (no block-level synchronisation).
#ifndef CHEMK_DI_WPB
#define CHEMK_DI_WPB 1
#endif
constexpr int kDiWavesPerBlock = CHEMK_DI_WPB;

__host__ __device__ inline int di_slice_doubles(int K, int R) {
    return (lds_doubles_per_wave(K, R, K + 1) + 1) & ~1;   // 16-byte aligned slices
}

// Persistent DI kernel: waves pull items from the queue until it is drained.
// NT: the register-resident LU's size (K + 1), or 0 for the LDS LU.
template <int NT>
__global__ void __launch_bounds__(64 * kDiWavesPerBlock) di_kernel(DevMech m, const int *__restrict__ n_items_p,
                                                const int *__restrict__ queue, int *counter,
                                                double *T, const double *p, double *Y,
                                                double dt, DIParams o, int *status,
                                                int *nsteps, unsigned long long *stats,
                                                int status_or) {
    extern __shared__ double lds[];
    const int wv = uniform((int)(threadIdx.x >> 6));   // wave index in the block, as a scalar
    const Lds L = carve_lds(lds + wv * di_slice_doubles(m.K, m.R), m.K, m.R, m.K + 1);
    const int lane = lane_id();
    const int K = m.K;
    const int n_items = *n_items_p;
    if (n_items <= 0) return;
    for (;;) {
        // Same-address atomics serialise in L2: a wave that reads the queue
        // as drained leaves without a claim (the claim below still decides;
        // this read only spares the final failing claims of every wave).
        if (uniform(__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >= n_items)
            break;
        // The claim is issued by every lane (lane 0 adds 1, the others 0) so
        // that no branch on the lane index precedes the broadcast of the
        // claimed index.  With a lane-0 branch here the compiler may thread
        // the previous iteration's lane-0 block straight into this one; lanes
        // 1..63 then reach the broadcast without lane 0, read their own zero
        // and never see the queue drain.
        const int got = atomicAdd(counter, lane == 0 ? 1 : 0);
        const int item = uniform(got);
        if (item >= n_items) break;
        const int c = queue ? queue[item] : item;
        double y = 0.0;
        if (lane < K) y = Y[(size_t)c * K + lane];
        else if (lane == K) y = T[c];
        int ns = 0;
        const int st = di_cell<NT>(m, L, p[c] * PA_TO_CGS, y, dt, o, ns);
        if (lane < K) Y[(size_t)c * K + lane] = y;
        else if (lane == K) T[c] = y;
        if (lane == 0) {
            status[c] = st | status_or;
            if (nsteps) nsteps[c] = ns;
        }
        // statistics: wave-level atomics with zero contributions off lane 0
        atomicAdd(&stats[1], lane == 0 ? (unsigned long long)ns : 0ull);
        atomicAdd(&stats[2], (lane == 0 && st != 0) ? 1ull : 0ull);
    }
}

// ---------------------------------------------------------------------------
// stiffness key, histogram and queue (binning)
// ---------------------------------------------------------------------------
// key = log10 of dt * max_k |dY_k/dt| / (|Y_k| + 1e-8) over the species, plus
// a temperature term; one wave per cell, one RHS evaluation.
__global__ void __launch_bounds__(64) stiffness_key_kernel(DevMech m, int n, const double *T,
                                                           const double *p, const double *Y,
                                                           double dt, int bins, int *bin_out) {
    extern __shared__ double lds[];
    const Lds L = carve_lds(lds, m.K, m.R, 1);
    const int lane = lane_id();
    const int K = m.K;
    for (int c = blockIdx.x; c < n; c += gridDim.x) {
        double y = 0.0;
        if (lane < K) y = Y[(size_t)c * K + lane];
        else if (lane == K) y = T[c];
        const double f = wave_rhs(m, L, p[c] * PA_TO_CGS, y);
        double act = lane < K ? fabs(f) * dt / (fabs(y) + 1e-8) : 0.0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) act = fmax(act, __shfl_xor(act, off, WAVE));
        if (lane == 0) {
            // map log10(activity) in [-6, 6] onto bins-1 .. 0 (bin 0 = most active)
            double lg = isfinite(act) ? log10(act + 1e-30) : 6.0;
            double x = (6.0 - lg) / 12.0 * bins;
            int b = (int)floor(x);
            b = b < 0 ? 0 : (b >= bins ? bins - 1 : b);
            bin_out[c] = b;
        }
    }
}

// The same key for the cells of a list: item i < *count is cell idx[i]
// (the DI fallback's routed cells, whose number only the device knows).
__global__ void __launch_bounds__(64) stiffness_key_list_kernel(DevMech m, const int *count, const int *idx,
                                                                const double *T, const double *p,
                                                                const double *Y, double dt, int bins,
                                                                int *bin_out) {
    extern __shared__ double lds[];
    const Lds L = carve_lds(lds, m.K, m.R, 1);
    const int lane = lane_id();
    const int K = m.K;
    const int cnt = uniform(*count);
    for (int i = blockIdx.x; i < cnt; i += gridDim.x) {
        const int c = uniform(idx[i]);
        double y = 0.0;
        if (lane < K) y = Y[(size_t)c * K + lane];
        else if (lane == K) y = T[c];
        const double f = wave_rhs(m, L, p[c] * PA_TO_CGS, y);
        double act = lane < K ? fabs(f) * dt / (fabs(y) + 1e-8) : 0.0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) act = fmax(act, __shfl_xor(act, off, WAVE));
        if (lane == 0) {
            double lg = isfinite(act) ? log10(act + 1e-30) : 6.0;
            double x = (6.0 - lg) / 12.0 * bins;
            int b = (int)floor(x);
            b = b < 0 ? 0 : (b >= bins ? bins - 1 : b);
            bin_out[i] = b;
        }
    }
}

__global__ void zero_ints_kernel(int *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void set_int_kernel(int *p, int v) { *p = v; }

__global__ void histogram_kernel(const int *bin, int n, int bins, int *hist) {
    __shared__ int h[256];
    for (int i = threadIdx.x; i < bins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        atomicAdd(&h[bin[i]], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < bins; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// exclusive scan of the histogram (bin 0 first); one thread.
__global__ void scan_kernel(const int *hist, int bins, int *offs) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int acc = 0;
        for (int b = 0; b < bins; ++b) {
            offs[b] = acc;
            acc += hist[b];
        }
    }
}

__global__ void histogram_list_kernel(const int *bin, const int *count, int bins, int *hist) {
    __shared__ int h[256];
    for (int i = threadIdx.x; i < bins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int n = *count;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        atomicAdd(&h[bin[i]], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < bins; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

__global__ void scatter_list_kernel(const int *bin, const int *count, int *offs, const int *idx,
                                    int *queue) {
    const int n = *count;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int pos = atomicAdd(&offs[bin[i]], 1);
        queue[pos] = idx[i];
    }
}

__global__ void scatter_kernel(const int *bin, int n, int *offs, int *queue) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int pos = atomicAdd(&offs[bin[i]], 1);
        queue[pos] = i;
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
int di_template_N(int Nreal) { return Nreal >= 2 && Nreal <= 64 ? Nreal : -1; }

// System sizes with a register-resident LU instance (N = K + 1 of the 9- and
// 32-species mechanisms).  A 54-column instance needs more than the 256
// architectural VGPRs; it agreed with the LDS LU bitwise in one build and not
// in the next (a change to code both paths share), with no cause found, so
// N = 54 takes the LDS LU.
bool di_has_reg_lu(int N) { return N == 10 || N == 33; }

size_t di_block_lds_bytes(int K, int R) {
    return sizeof(double) * (size_t)di_slice_doubles(K, R) * kDiWavesPerBlock;
}

size_t di_lds_bytes(int K, int R, int N) {
    return sizeof(double) * (size_t)lds_doubles_per_wave(K, R, N);
}

hipError_t launch_di(const DevMech &m, int grid, const int *n_items, const int *queue,
                     int *counter, double *T, const double *p, double *Y, double dt,
                     double rtol, double atolY, double atolT, double h0_frac, int max_steps,
                     int project, int *status, int *nsteps, unsigned long long *stats,
                     int status_or, int variant, hipStream_t s) {
    DIParams o{rtol, atolY, atolT, h0_frac, max_steps, project};
    const size_t lds = di_block_lds_bytes(m.K, m.R);
    const int blocks = (grid + kDiWavesPerBlock - 1) / kDiWavesPerBlock;
    const bool reg = variant != CHEMK_DI_LDS_LU && di_has_reg_lu(m.N);
    if (variant == CHEMK_DI_REG_LU && !reg) return hipErrorInvalidValue;
#define CHEMK_LAUNCH_DI(NT)                                                                    \
    hipLaunchKernelGGL(di_kernel<NT>, dim3(blocks), dim3(64 * kDiWavesPerBlock), lds, s, m,    \
                       n_items, queue, counter, T, p, Y, dt, o, status, nsteps, stats, status_or)
    if (!reg) CHEMK_LAUNCH_DI(0);
    else if (m.N == 10) CHEMK_LAUNCH_DI(10);
    else CHEMK_LAUNCH_DI(33);
#undef CHEMK_LAUNCH_DI
    return hipGetLastError();
}

hipError_t launch_binning(const DevMech &m, int n, const double *T, const double *p,
                          const double *Y, double dt, int bins, int *bin, int *hist, int *offs,
                          int *queue, hipStream_t s) {
    const size_t lds = di_lds_bytes(m.K, m.R, 1);
    const int grid_key = n < 8192 ? n : 8192;
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(256), 0, s, hist, bins);
    hipLaunchKernelGGL(stiffness_key_kernel, dim3(grid_key), dim3(64), lds, s, m, n, T, p, Y, dt,
                       bins, bin);
    const int g = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;
    hipLaunchKernelGGL(histogram_kernel, dim3(g), dim3(256), 0, s, bin, n, bins, hist);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(64), 0, s, hist, bins, offs);
    hipLaunchKernelGGL(scatter_kernel, dim3(g), dim3(256), 0, s, bin, n, offs, queue);
    return hipGetLastError();
}

hipError_t launch_binning_list(const DevMech &m, int n_max, const int *count, const int *idx,
                               const double *T, const double *p, const double *Y, double dt, int bins,
                               int *bin, int *hist, int *offs, int *queue, hipStream_t s) {
    if (n_max <= 0) return hipSuccess;
    const size_t lds = di_lds_bytes(m.K, m.R, 1);
    const int grid_key = n_max < 8192 ? n_max : 8192;
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(256), 0, s, hist, bins);
    hipLaunchKernelGGL(stiffness_key_list_kernel, dim3(grid_key), dim3(64), lds, s, m, count, idx, T, p, Y,
                       dt, bins, bin);
    const int g = (n_max + 255) / 256 < 1024 ? (n_max + 255) / 256 : 1024;
    hipLaunchKernelGGL(histogram_list_kernel, dim3(g), dim3(256), 0, s, bin, count, bins, hist);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(64), 0, s, hist, bins, offs);
    hipLaunchKernelGGL(scatter_list_kernel, dim3(g), dim3(256), 0, s, bin, count, offs, idx, queue);
    return hipGetLastError();
}

hipError_t launch_zero_ints(int *p, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_set_int(int *p, int v, hipStream_t s) {
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

}  // namespace chemk
