/*
 * chem_oracle.c -- plain, slow FP64 CPU reference of the per-cell chemistry
 * advance.  TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the GPU library never
 * does and shares no code, header or table with it.
 *
 * What it computes (the paper, Sec. II.B, Eqs. 1-2): the ODE system
 * dy/dt = phi(y; p) for y = (Y_1..Y_K, T) at constant pressure, integrated over
 * one flow step dt for every cell independently, giving the pair
 * phi(t) => phi(t+dt).  The paper leaves the rate laws to its mechanism; the
 * laws written out here are the textbook ones the workload specifies:
 *   - ideal gas, mixture molar mass Wbar = 1/sum(Y_k/W_k), rho = p Wbar/(R_u T);
 *   - NASA-7 polynomials (single range) for cp, h, s of each species;
 *   - mass action with modified Arrhenius k_f = A T^b exp(-Ea/(R_c T)) in cgs
 *     units, reverse rates k_r = k_f/K_c with K_c = K_p (p0/(R_u T))^dnu from
 *     the Gibbs energies, third bodies with unit efficiencies ([M] = p/(R_u T));
 *   - dY_k/dt = W_k omega_k / rho and the constant-pressure energy equation
 *     dT/dt = -sum_k H_k omega_k / (rho cp);
 *   - the temperature after the step is recovered from the conserved mixture
 *     enthalpy by Newton's method on the NASA polynomials (the property update
 *     of Sec. II.A uses Newton's method and temperature polynomials).
 * Integration: RODAS (Hairer & Wanner, Solving ODEs II, Sec. VI.4), the
 * 6-stage stiffly accurate Rosenbrock method of order 4 with an embedded
 * order-3 solution, in its W-transformed form, with dense LU and partial
 * pivoting; step-size control by the weighted RMS norm of the embedded error.
 *
 * Units: SI except rate constants and concentrations inside the rate law,
 * which are cgs (mol/cm^3, cm^3/mol/s); Ea in cal/mol; W in g/mol.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_RU 8.31446261815324            /* J/(mol K) */
#define OR_RC (OR_RU / 4.184)             /* cal/(mol K) */
#define OR_PSTD 101325.0                  /* standard-state pressure, Pa */
#define OR_MAXK 64
#define OR_MAXN (OR_MAXK + 1)

typedef struct {
    int32_t E, K, R;
    const double *emass;     /* [E] g/mol */
    const int32_t *comp;     /* [K*E] atoms of element e in species k */
    const double *nasa;      /* [K*7] */
    const int32_t *reac;     /* [R*2], -1 = empty */
    const int32_t *prod;     /* [R*2], -1 = empty */
    const double *lnA;       /* [R] ln A, cgs */
    const double *beta;      /* [R] */
    const double *Ea;        /* [R] cal/mol */
    const int32_t *tb;       /* [R] third body flag */
    const int32_t *rev;      /* [R] reversible flag */
} or_mech;

/* -------------------------------------------------------------------- */
/* thermodynamics                                                        */
/* -------------------------------------------------------------------- */

double or_molar_mass(const or_mech *m, int k)
{
    double w = 0.0;
    for (int e = 0; e < m->E; ++e) w += m->comp[k * m->E + e] * m->emass[e];
    return w;
}

/* NASA-7: cp/R, h/(RT), s/R of species k at temperature T. */
void or_species_thermo(const or_mech *m, double T, double *cpR, double *hRT, double *sR)
{
    for (int k = 0; k < m->K; ++k) {
        const double *a = m->nasa + 7 * k;
        cpR[k] = a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T;
        hRT[k] = a[0] + a[1] * T / 2 + a[2] * T * T / 3 + a[3] * T * T * T / 4
               + a[4] * T * T * T * T / 5 + a[5] / T;
        sR[k] = a[0] * log(T) + a[1] * T + a[2] * T * T / 2 + a[3] * T * T * T / 3
              + a[4] * T * T * T * T / 4 + a[6];
    }
}

/* d(cp/R)/dT of species k. */
static double species_dcpR_dT(const or_mech *m, int k, double T)
{
    const double *a = m->nasa + 7 * k;
    return a[1] + 2 * a[2] * T + 3 * a[3] * T * T + 4 * a[4] * T * T * T;
}

/* mass-specific mixture cp [J/(kg K)] and h [J/kg]. */
void or_mixture_cp_h(const or_mech *m, double T, const double *Y, double *cp, double *h)
{
    double cpR[OR_MAXK], hRT[OR_MAXK], sR[OR_MAXK];
    or_species_thermo(m, T, cpR, hRT, sR);
    double c = 0.0, hh = 0.0;
    for (int k = 0; k < m->K; ++k) {
        double Wkg = or_molar_mass(m, k) * 1e-3;
        c += Y[k] * cpR[k] * OR_RU / Wkg;
        hh += Y[k] * hRT[k] * OR_RU * T / Wkg;
    }
    *cp = c;
    *h = hh;
}

/* -------------------------------------------------------------------- */
/* kinetics                                                              */
/* -------------------------------------------------------------------- */

typedef struct {
    double rho;               /* kg/m^3 */
    double Wbar;              /* g/mol */
    double M;                 /* third-body concentration, mol/cm^3 */
    double C[OR_MAXK];        /* mol/cm^3 */
    double cpR[OR_MAXK], hRT[OR_MAXK], sR[OR_MAXK];
} or_state;

static void state_eval(const or_mech *m, double T, double p, const double *Y, or_state *s)
{
    double sum = 0.0;
    for (int k = 0; k < m->K; ++k) sum += Y[k] / or_molar_mass(m, k);
    s->Wbar = 1.0 / sum;
    s->rho = p * s->Wbar * 1e-3 / (OR_RU * T);
    for (int k = 0; k < m->K; ++k)
        s->C[k] = s->rho * Y[k] / (or_molar_mass(m, k) * 1e-3) * 1e-6;
    s->M = p / (OR_RU * T) * 1e-6;
    or_species_thermo(m, T, s->cpR, s->hRT, s->sR);
}

static int n_slots(const int32_t *v) { return (v[0] >= 0) + (v[1] >= 0); }

/* Rate constants of reaction j: k_f, k_r (cgs). */
static void rate_constants(const or_mech *m, const or_state *s, double T, int j,
                           double *kf, double *kr)
{
    *kf = exp(m->lnA[j] + m->beta[j] * log(T) - m->Ea[j] / (OR_RC * T));
    if (!m->rev[j]) {
        *kr = 0.0;
        return;
    }
    double dg = 0.0; /* sum nu_k g_k/RT */
    for (int i = 0; i < 2; ++i) {
        int a = m->reac[2 * j + i], b = m->prod[2 * j + i];
        if (a >= 0) dg -= s->hRT[a] - s->sR[a];
        if (b >= 0) dg += s->hRT[b] - s->sR[b];
    }
    int dnu = n_slots(m->prod + 2 * j) - n_slots(m->reac + 2 * j);
    double lnKc = -dg + dnu * log(OR_PSTD / (OR_RU * T) * 1e-6);
    *kr = *kf / exp(lnKc);
}

/* Forward and reverse fluxes of every reaction (mol/cm^3/s). */
void or_fluxes(const or_mech *m, double T, double p, const double *Y, double *qf, double *qr)
{
    or_state s;
    state_eval(m, T, p, Y, &s);
    for (int j = 0; j < m->R; ++j) {
        double kf, kr;
        rate_constants(m, &s, T, j, &kf, &kr);
        double f = kf, r = kr;
        for (int i = 0; i < 2; ++i) {
            int a = m->reac[2 * j + i], b = m->prod[2 * j + i];
            if (a >= 0) f *= s.C[a];
            if (b >= 0) r *= s.C[b];
        }
        if (m->tb[j]) {
            f *= s.M;
            r *= s.M;
        }
        qf[j] = f;
        qr[j] = r;
    }
}

/* Type of the rate products and production rates in the right-hand side.
 * The oracle is FP64 throughout; a test compiles a variant with
 * -DOR_RATE_T=float (rate constants still from FP64 exp/log, Jacobian, LU and
 * error control still FP64) to measure what FP32 rate evaluation costs. */
#ifndef OR_RATE_T
#define OR_RATE_T double
#endif

/* Right-hand side f(y), y = (Y_1..Y_K, T), constant p. */
void or_rhs(const or_mech *m, double p, const double *y, double *f)
{
    const int K = m->K;
    double T = y[K];
    or_state s;
    state_eval(m, T, p, y, &s);
    OR_RATE_T omega[OR_MAXK];
    for (int k = 0; k < K; ++k) omega[k] = 0;
    for (int j = 0; j < m->R; ++j) {
        double kf, kr;
        rate_constants(m, &s, T, j, &kf, &kr);
        OR_RATE_T fw = (OR_RATE_T)kf, rv = (OR_RATE_T)kr;
        for (int i = 0; i < 2; ++i) {
            int a = m->reac[2 * j + i], b = m->prod[2 * j + i];
            if (a >= 0) fw *= (OR_RATE_T)s.C[a];
            if (b >= 0) rv *= (OR_RATE_T)s.C[b];
        }
        OR_RATE_T q = fw - rv;
        if (m->tb[j]) q *= (OR_RATE_T)s.M;
        for (int i = 0; i < 2; ++i) {
            int a = m->reac[2 * j + i], b = m->prod[2 * j + i];
            if (a >= 0) omega[a] -= q;
            if (b >= 0) omega[b] += q;
        }
    }
    double cp = 0.0, hw = 0.0;
    for (int k = 0; k < K; ++k) {
        double Wkg = or_molar_mass(m, k) * 1e-3;
        double w = omega[k] * 1e6;                      /* mol/m^3/s */
        f[k] = Wkg * w / s.rho;
        cp += y[k] * s.cpR[k] * OR_RU / Wkg;
        hw += s.hRT[k] * OR_RU * T * w;
    }
    f[K] = -hw / (s.rho * cp);
}

/* Analytic Jacobian J[i*N+j] = d f_i / d y_j, N = K+1, written term by term:
 * concentrations C_i = rho Y_i / W_i with rho = p Wbar/(R_u T), so
 *   dC_i/dY_j = delta_ij rho/W_i + (Y_i/W_i) drho/dY_j,  drho/dY_j = -rho Wbar/W_j,
 *   dC_i/dT   = -C_i / T;
 * dq/dC from mass action, dq/dT from k_f, k_r and [M] at fixed C.           */
void or_jacobian(const or_mech *m, double p, const double *y, double *J)
{
    const int K = m->K, N = K + 1;
    const double T = y[K];
    or_state s;
    state_eval(m, T, p, y, &s);
    double W[OR_MAXK];
    for (int k = 0; k < K; ++k) W[k] = or_molar_mass(m, k) * 1e-3;   /* kg/mol */

    /* concentrations in SI (mol/m^3) for the chain rule */
    double Csi[OR_MAXK];
    for (int k = 0; k < K; ++k) Csi[k] = s.C[k] * 1e6;
    double drho_dY[OR_MAXK];
    for (int j = 0; j < K; ++j) drho_dY[j] = -s.rho * (s.Wbar * 1e-3) / W[j];
    double drho_dT = -s.rho / T;

    /* domega_k/dY_j (SI) and domega_k/dT */
    static __thread double dwdY[OR_MAXK * OR_MAXK];
    double dwdT[OR_MAXK], omega[OR_MAXK];
    memset(dwdY, 0, sizeof(double) * K * K);
    for (int k = 0; k < K; ++k) dwdT[k] = omega[k] = 0.0;

    for (int r = 0; r < m->R; ++r) {
        double kf, kr;
        rate_constants(m, &s, T, r, &kf, &kr);
        /* forward / reverse products of concentrations (SI) */
        double Mf = m->tb[r] ? s.M * 1e6 : 1.0;
        /* convert rate constants to SI: factor 1e-6 per concentration beyond the first */
        int nr = n_slots(m->reac + 2 * r), np = n_slots(m->prod + 2 * r);
        int ordf = nr + (m->tb[r] ? 1 : 0), ordr = np + (m->tb[r] ? 1 : 0);
        double kfs = kf * pow(1e-6, ordf - 1);
        double krs = kr * pow(1e-6, ordr - 1);
        double pf = kfs * Mf, pr = krs * Mf;
        for (int i = 0; i < 2; ++i) {
            int a = m->reac[2 * r + i], b = m->prod[2 * r + i];
            if (a >= 0) pf *= Csi[a];
            if (b >= 0) pr *= Csi[b];
        }
        double q = pf - pr;
        /* dq/dC_i (SI) */
        double dqdC[OR_MAXK];
        for (int k = 0; k < K; ++k) dqdC[k] = 0.0;
        for (int i = 0; i < 2; ++i) {
            int a = m->reac[2 * r + i];
            if (a < 0) continue;
            double prodo = kfs * Mf;
            for (int i2 = 0; i2 < 2; ++i2) {
                int a2 = m->reac[2 * r + i2];
                if (i2 != i && a2 >= 0) prodo *= Csi[a2];
            }
            dqdC[a] += prodo;
        }
        for (int i = 0; i < 2; ++i) {
            int b = m->prod[2 * r + i];
            if (b < 0) continue;
            double prodo = krs * Mf;
            for (int i2 = 0; i2 < 2; ++i2) {
                int b2 = m->prod[2 * r + i2];
                if (i2 != i && b2 >= 0) prodo *= Csi[b2];
            }
            dqdC[b] -= prodo;
        }
        /* dq/dT at fixed C */
        double dlnkf = m->beta[r] / T + m->Ea[r] / (OR_RC * T * T);
        double dlnKc = 0.0;
        if (m->rev[r]) {
            for (int i = 0; i < 2; ++i) {
                int a = m->reac[2 * r + i], b = m->prod[2 * r + i];
                if (a >= 0) dlnKc -= s.hRT[a] / T;
                if (b >= 0) dlnKc += s.hRT[b] / T;
            }
            dlnKc -= (np - nr) / T;
        }
        double dlnM = m->tb[r] ? -1.0 / T : 0.0;
        double dqdT_C = pf * (dlnkf + dlnM) - pr * (dlnkf - dlnKc + dlnM);

        /* stoichiometric coefficients of this reaction */
        double nu[OR_MAXK];
        for (int k = 0; k < K; ++k) nu[k] = 0.0;
        for (int i = 0; i < 2; ++i) {
            int a = m->reac[2 * r + i], b = m->prod[2 * r + i];
            if (a >= 0) nu[a] -= 1.0;
            if (b >= 0) nu[b] += 1.0;
        }
        /* dq/dY_j = sum_i dq/dC_i dC_i/dY_j ; dq/dT = dq/dT|_C + sum_i dq/dC_i dC_i/dT */
        double dqdY[OR_MAXK];
        double dqdT = dqdT_C;
        for (int j = 0; j < K; ++j) {
            double acc = 0.0;
            for (int i = 0; i < K; ++i) {
                double dCdY = (i == j ? s.rho / W[i] : 0.0) + y[i] / W[i] * drho_dY[j];
                acc += dqdC[i] * dCdY;
            }
            dqdY[j] = acc;
        }
        for (int i = 0; i < K; ++i) dqdT += dqdC[i] * (-Csi[i] / T);
        for (int k = 0; k < K; ++k) {
            if (nu[k] == 0.0) continue;
            omega[k] += nu[k] * q;
            dwdT[k] += nu[k] * dqdT;
            for (int j = 0; j < K; ++j) dwdY[k * K + j] += nu[k] * dqdY[j];
        }
    }

    /* species rows: f_k = W_k omega_k / rho */
    for (int k = 0; k < K; ++k) {
        for (int j = 0; j < K; ++j)
            J[k * N + j] = W[k] * dwdY[k * K + j] / s.rho
                         - W[k] * omega[k] / (s.rho * s.rho) * drho_dY[j];
        J[k * N + K] = W[k] * dwdT[k] / s.rho - W[k] * omega[k] / (s.rho * s.rho) * drho_dT;
    }
    /* temperature row: f_T = -sum_k H_k omega_k / (rho cp) */
    double cp = 0.0, dcpdT = 0.0, Hw = 0.0;
    double cpk[OR_MAXK], Hk[OR_MAXK];
    for (int k = 0; k < K; ++k) {
        cpk[k] = s.cpR[k] * OR_RU / W[k];                /* J/(kg K) */
        Hk[k] = s.hRT[k] * OR_RU * T;                    /* J/mol */
        cp += y[k] * cpk[k];
        dcpdT += y[k] * species_dcpR_dT(m, k, T) * OR_RU / W[k];
        Hw += Hk[k] * omega[k];
    }
    double D = s.rho * cp;
    for (int j = 0; j < K; ++j) {
        double num = 0.0;
        for (int k = 0; k < K; ++k) num += Hk[k] * dwdY[k * K + j];
        double dD = cp * drho_dY[j] + s.rho * cpk[j];
        J[K * N + j] = -num / D + Hw / (D * D) * dD;
    }
    {
        double num = 0.0;
        for (int k = 0; k < K; ++k) num += s.cpR[k] * OR_RU * omega[k] + Hk[k] * dwdT[k];
        double dD = cp * drho_dT + s.rho * dcpdT;
        J[K * N + K] = -num / D + Hw / (D * D) * dD;
    }
}

/* -------------------------------------------------------------------- */
/* dense LU with partial pivoting (ties keep the lowest row index)       */
/* -------------------------------------------------------------------- */

int or_lu(int n, double *A, int *piv)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > best) {
                best = fabs(A[i * n + k]);
                p = i;
            }
        piv[k] = p;
        if (best == 0.0) return -1;
        if (p != k)
            for (int j = 0; j < n; ++j) {
                double t = A[k * n + j];
                A[k * n + j] = A[p * n + j];
                A[p * n + j] = t;
            }
        for (int i = k + 1; i < n; ++i) {
            double l = A[i * n + k] / A[k * n + k];
            A[i * n + k] = l;
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
        }
    }
    return 0;
}

void or_lu_solve(int n, const double *LU, const int *piv, double *b)
{
    for (int k = 0; k < n; ++k) {
        int p = piv[k];
        if (p != k) {
            double t = b[k];
            b[k] = b[p];
            b[p] = t;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) b[i] -= LU[i * n + j] * b[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) b[i] -= LU[i * n + j] * b[j];
        b[i] /= LU[i * n + i];
    }
}

/* -------------------------------------------------------------------- */
/* RODAS (Hairer & Wanner), transformed form:                            */
/*   (1/(h g) I - J) u_i = f(y0 + sum_j a_ij u_j) + sum_j (c_ij/h) u_j    */
/*   y1 = y0 + a51 u1 + .. + a54 u4 + u5 + u6, error estimate = u6.       */
/* -------------------------------------------------------------------- */

typedef void (*or_fun)(void *ctx, const double *y, double *f);

static const double RG = 0.25;
static const double RA[6][5] = {
    {0, 0, 0, 0, 0},
    {1.544, 0, 0, 0, 0},
    {0.9466785280815826, 0.2557011698983284, 0, 0, 0},
    {3.314825187068521, 2.896124015972201, 0.9986419139977817, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0}};
static const double RC_[6][5] = {
    {0, 0, 0, 0, 0},
    {-5.6688, 0, 0, 0, 0},
    {-2.430093356833875, -0.2063599157091915, 0, 0, 0},
    {-0.1073529058151375, -9.594562251023355, -20.47028614809616, 0, 0},
    {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.70890893206160, 0},
    {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136,
     -6.058818238834054}};

/* Coefficients exported for the order-condition test. */
void or_rodas_coefficients(double *gamma, double *A, double *C)
{
    *gamma = RG;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 5; ++j) {
            A[i * 5 + j] = RA[i][j];
            C[i * 5 + j] = RC_[i][j];
        }
}

typedef struct {
    int nsteps, naccept, nreject;
    double h_last;
} or_stats;

/* Integrate y over [0, tend].  fixed_h > 0 disables step control (order tests).
 * Returns 0 ok, 1 too many steps / step underflow, 3 non-finite, 6 singular.  */
int or_rodas(int N, or_fun f, or_fun jac, void *ctx, double *y, double tend,
             const double *atol, double rtol, double h0, int max_steps,
             double fixed_h, or_stats *st)
{
    double J[OR_MAXN * OR_MAXN], A[OR_MAXN * OR_MAXN];
    int piv[OR_MAXN];
    double f0[OR_MAXN], fy[OR_MAXN], yt[OR_MAXN], u[6][OR_MAXN], ynew[OR_MAXN];
    double t = 0.0, h = fixed_h > 0 ? fixed_h : h0;
    int need_jac = 1, rejected = 0;
    st->nsteps = st->naccept = st->nreject = 0;
    f(ctx, y, f0);
    while (t < tend) {
        if (st->nsteps >= max_steps) return 1;
        int last = 0;
        if (t + h >= tend * (1.0 - 1e-14) || t + h >= tend) {
            h = tend - t;
            last = 1;
        }
        if (h <= 1e-14 * tend * 1e-6 || h <= 0.0) return 1;
        if (need_jac) {
            jac(ctx, y, J);
            need_jac = 0;
        }
        st->nsteps++;
        double fac = 1.0 / (h * RG);
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) A[i * N + j] = (i == j ? fac : 0.0) - J[i * N + j];
        if (or_lu(N, A, piv)) return 6;
        for (int s = 0; s < 6; ++s) {
            const double *fs;
            if (s == 0) {
                fs = f0;
            } else {
                for (int i = 0; i < N; ++i) {
                    double acc = y[i];
                    for (int j = 0; j < s; ++j) acc += RA[s][j] * u[j][i];
                    yt[i] = acc;
                }
                f(ctx, yt, fy);
                fs = fy;
            }
            for (int i = 0; i < N; ++i) {
                double acc = fs[i];
                for (int j = 0; j < s; ++j) acc += RC_[s][j] / h * u[j][i];
                u[s][i] = acc;
            }
            or_lu_solve(N, A, piv, u[s]);
        }
        double err = 0.0;
        int finite = 1;
        for (int i = 0; i < N; ++i) {
            ynew[i] = yt[i] + u[5][i];
            double sc = atol[i] + rtol * fmax(fabs(y[i]), fabs(ynew[i]));
            double e = u[5][i] / sc;
            err += e * e;
            if (!isfinite(ynew[i])) finite = 0;
        }
        err = sqrt(err / N);
        if (!finite || !isfinite(err)) {
            if (fixed_h > 0) return 3;
            /* treat as a rejection with the largest reduction */
            h *= 0.2;
            rejected = 1;
            st->nreject++;
            continue;
        }
        if (fixed_h > 0 || err <= 1.0) {
            t = last ? tend : t + h;
            memcpy(y, ynew, sizeof(double) * N);
            f(ctx, y, f0);
            need_jac = 1;
            st->naccept++;
            if (fixed_h <= 0) {
                double fc = err > 0 ? 0.9 / sqrt(sqrt(err)) : 5.0;
                fc = fmin(5.0, fmax(0.2, fc));
                if (rejected) fc = fmin(fc, 1.0);
                h *= fc;
            }
            rejected = 0;
        } else {
            double fc = fmax(0.2, 0.9 / sqrt(sqrt(err)));
            h *= fc;
            rejected = 1;
            st->nreject++;
        }
    }
    st->h_last = h;
    return 0;
}

/* -------------------------------------------------------------------- */
/* temperature from enthalpy, element projection, cell driver             */
/* -------------------------------------------------------------------- */

/* Newton on h(T) = h0 (tolerance 1e-12 relative, at most 50 iterations),
 * bisection on [200, 4000] K if Newton fails.  Returns 0 ok, 4 failure. */
int or_T_from_h(const or_mech *m, double h0, const double *Y, double T_guess, double *T_out)
{
    double T = T_guess;
    for (int it = 0; it < 50; ++it) {
        double cp, h;
        or_mixture_cp_h(m, T, Y, &cp, &h);
        double dT = (h - h0) / cp;
        T -= dT;
        if (!isfinite(T)) break;
        if (fabs(dT) <= 1e-12 * fabs(T)) {
            if (T >= 200.0 && T <= 4000.0) {
                *T_out = T;
                return 0;
            }
            break;
        }
    }
    double lo = 200.0, hi = 4000.0, cp, hlo, hhi;
    or_mixture_cp_h(m, lo, Y, &cp, &hlo);
    or_mixture_cp_h(m, hi, Y, &cp, &hhi);
    if (!(hlo <= h0 && h0 <= hhi)) {
        *T_out = T_guess;
        return 4;
    }
    for (int it = 0; it < 200 && hi - lo > 1e-13 * hi; ++it) {
        double mid = 0.5 * (lo + hi), hm;
        or_mixture_cp_h(m, mid, Y, &cp, &hm);
        if (hm < h0) lo = mid;
        else hi = mid;
    }
    *T_out = 0.5 * (lo + hi);
    return 0;
}

/* Element mass fractions m_e = sum_k Y_k n_ek A_e / W_k. */
void or_element_mass(const or_mech *m, const double *Y, double *me)
{
    for (int e = 0; e < m->E; ++e) {
        double acc = 0.0;
        for (int k = 0; k < m->K; ++k)
            acc += Y[k] * m->comp[k * m->E + e] * m->emass[e] / or_molar_mass(m, k);
        me[e] = acc;
    }
}

/* Minimum-norm (weights w_k = max(Y_k, 1e-30)) correction of Y so that its
 * element masses equal those of Yref:  Y <- Y - W E^T (E W E^T)^-1 (E Y - E Yref). */
void or_project(const or_mech *m, const double *Yref, double *Y)
{
    const int E = m->E, K = m->K;
    double mr[8], my[8], A[64], lam[8];
    int piv[8];
    or_element_mass(m, Yref, mr);
    or_element_mass(m, Y, my);
    double Em[8 * OR_MAXK], w[OR_MAXK];
    for (int k = 0; k < K; ++k) {
        w[k] = Y[k] > 1e-30 ? Y[k] : 1e-30;
        for (int e = 0; e < E; ++e)
            Em[e * K + k] = m->comp[k * E + e] * m->emass[e] / or_molar_mass(m, k);
    }
    for (int a = 0; a < E; ++a) {
        lam[a] = my[a] - mr[a];
        for (int b = 0; b < E; ++b) {
            double acc = 0.0;
            for (int k = 0; k < K; ++k) acc += Em[a * K + k] * w[k] * Em[b * K + k];
            A[a * E + b] = acc;
        }
    }
    if (or_lu(E, A, piv)) return;
    or_lu_solve(E, A, piv, lam);
    for (int k = 0; k < K; ++k) {
        double acc = 0.0;
        for (int e = 0; e < E; ++e) acc += Em[e * K + k] * lam[e];
        Y[k] -= w[k] * acc;
    }
}

typedef struct {
    const or_mech *m;
    double p;
} chem_ctx;

static void chem_f(void *c, const double *y, double *f)
{
    chem_ctx *cc = (chem_ctx *)c;
    or_rhs(cc->m, cc->p, y, f);
}

static void chem_j(void *c, const double *y, double *J)
{
    chem_ctx *cc = (chem_ctx *)c;
    or_jacobian(cc->m, cc->p, y, J);
}

/* Options of the cell advance. */
typedef struct {
    double rtol, atol_Y, atol_T;
    double h0_frac;         /* first trial step = h0_frac * dt */
    int32_t max_steps;
    int32_t project;        /* element projection of the final Y */
    int32_t newton_T;       /* final T from the conserved enthalpy */
} or_opts;

/* Advance one cell; status 0 ok, 1 steps, 2 T range, 3 non-finite, 4 Newton, 6 singular. */
int or_advance_cell(const or_mech *m, double *T, double p, double *Y, double dt,
                    const or_opts *o, or_stats *st)
{
    const int K = m->K, N = K + 1;
    double y[OR_MAXN], Yin[OR_MAXK], atol[OR_MAXN], cp, h0;
    for (int k = 0; k < K; ++k) {
        y[k] = Yin[k] = Y[k];
        atol[k] = o->atol_Y;
    }
    y[K] = *T;
    atol[K] = o->atol_T;
    or_mixture_cp_h(m, *T, Y, &cp, &h0);
    chem_ctx c = {m, p};
    int rc = or_rodas(N, chem_f, chem_j, &c, y, dt, atol, o->rtol, o->h0_frac * dt,
                      o->max_steps, 0.0, st);
    for (int i = 0; i < N; ++i)
        if (!isfinite(y[i])) rc = rc ? rc : 3;
    if (rc) return rc;
    if (o->project) or_project(m, Yin, y);
    double Tn = y[K];
    if (o->newton_T) {
        if (or_T_from_h(m, h0, y, y[K], &Tn)) return 4;
    }
    for (int k = 0; k < K; ++k) Y[k] = y[k];
    *T = Tn;
    if (Tn < 200.0 || Tn > 4000.0) return 2;
    return 0;
}

/* All cells, OpenMP over cells (dynamic schedule, one cell at a time: a cell
 * costs milliseconds, so the scheduling overhead is negligible). */
void or_advance(const or_mech *m, int64_t n, double *T, const double *p, double *Y,
                double dt, const or_opts *o, int32_t *status, int32_t *nsteps, int nthreads)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t c = 0; c < n; ++c) {
        or_stats st = {0, 0, 0, 0.0};
        status[c] = or_advance_cell(m, T + c, p[c], Y + c * m->K, dt, o, &st);
        if (nsteps) nsteps[c] = st.nsteps;
    }
}

/* Batched property evaluations (for parity of the property kernels). */
void or_thermo_batch(const or_mech *m, int64_t n, const double *T, const double *Y,
                     double *cp, double *h)
{
    for (int64_t c = 0; c < n; ++c) or_mixture_cp_h(m, T[c], Y + c * m->K, cp + c, h + c);
}

void or_T_from_h_batch(const or_mech *m, int64_t n, const double *h, const double *Y,
                       double *T, int32_t *status)
{
    for (int64_t c = 0; c < n; ++c) {
        double Tout;
        status[c] = or_T_from_h(m, h[c], Y + c * m->K, T[c], &Tout);
        T[c] = Tout;
    }
}

void or_rhs_batch(const or_mech *m, int64_t n, const double *T, const double *p,
                  const double *Y, double *f)
{
    const int K = m->K, N = K + 1;
    for (int64_t c = 0; c < n; ++c) {
        double y[OR_MAXN];
        for (int k = 0; k < K; ++k) y[k] = Y[c * K + k];
        y[K] = T[c];
        or_rhs(m, p[c], y, f + c * N);
    }
}

void or_jacobian_batch(const or_mech *m, int64_t n, const double *T, const double *p,
                       const double *Y, double *J)
{
    const int K = m->K, N = K + 1;
    for (int64_t c = 0; c < n; ++c) {
        double y[OR_MAXN];
        for (int k = 0; k < K; ++k) y[k] = Y[c * K + k];
        y[K] = T[c];
        or_jacobian(m, p[c], y, J + c * N * N);
    }
}

/* Generic RODAS on caller-supplied callbacks (integrator pins on test ODEs). */
int or_rodas_generic(int N, or_fun f, or_fun jac, double *y, double tend, const double *atol,
                     double rtol, double h0, int max_steps, double fixed_h, int32_t *counts)
{
    or_stats st;
    int rc = or_rodas(N, f, jac, NULL, y, tend, atol, rtol, h0, max_steps, fixed_h, &st);
    counts[0] = st.nsteps;
    counts[1] = st.naccept;
    counts[2] = st.nreject;
    return rc;
}
