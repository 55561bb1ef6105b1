/*
 * chemk.h -- C ABI of the MI355X (gfx950) chemistry-advance library.
 *
 * The library advances the thermochemical state (T, p, Y_1..Y_K) of every
 * cell of a reacting-flow solver over one flow time step dt, either by direct
 * integration (DI) of the stiff kinetics ODEs or by a multilayer perceptron
 * that stands in for DI, and evaluates the thermal properties around that
 * step.  This is the chemistry part of the GPU-ANN LES method of Zhang et al.
 * (Sec. II): the ODE system of Eq. 1, integrated over a step to give the pair
 * of Eq. 2 per cell; the ANN replacement of Sec. II.A/II.B (inputs {T, p,
 * F(Y)}, output Y(t+dt) - Y(t), Box-Cox transform of Eq. 7, GELU MLP trained
 * with Adam on the loss of Eq. 8); and the property update of Sec. II.A
 * (temperature from enthalpy by Newton's method on temperature polynomials).
 *
 * Conventions shared by every call:
 *  - All state arrays are caller-owned DEVICE memory on the context's GPU,
 *    FP64 unless stated, and must stay valid until the work enqueued on
 *    `stream` has completed.  Y is row-major (n, K): Y[c*K + k].
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls are asynchronous: CHEMK_OK means "validated and enqueued".  The
 *    library never synchronises unless a call says so.
 *  - Host-side argument checks run before anything is enqueued; on error
 *    nothing is enqueued, outputs are untouched and chemk_last_error()
 *    returns a message (thread-local, valid until the next call on the
 *    same thread).
 *  - Units: SI for T [K], p [Pa], h [J/kg], cp [J/(kg K)], time [s]; the
 *    mechanism's rate parameters are cgs (mol, cm, s) with Ea in cal/mol.
 */
#ifndef CHEMK_H
#define CHEMK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
enum {
    CHEMK_OK = 0,
    CHEMK_E_ARG = 1,          /* bad argument (null pointer, size, option)        */
    CHEMK_E_MECH = 2,         /* mechanism rejected (not element-conserving, ...) */
    CHEMK_E_HIP = 3,          /* HIP runtime error                                 */
    CHEMK_E_DT = 4,           /* ANN advance with a dt other than the trained one  */
    CHEMK_E_OOM = 5,          /* device allocation failed                          */
    CHEMK_E_STATE = 6,        /* call out of order (e.g. ANN used before set-up)   */
    CHEMK_E_UNSUPPORTED = 7   /* size outside what the kernels support             */
};

/* ---- per-cell outcome codes written to `status` -------------------------- */
enum {
    CHEMK_CELL_OK = 0,
    CHEMK_CELL_MAX_STEPS = 1, /* integrator hit max_steps or a step underflow     */
    CHEMK_CELL_T_RANGE = 2,   /* final T outside [200, 4000] K                    */
    CHEMK_CELL_NONFINITE = 3, /* non-finite state                                 */
    CHEMK_CELL_NEWTON = 4,    /* T from enthalpy failed (h outside the T range)    */
    CHEMK_CELL_SINGULAR = 6,  /* singular iteration matrix                        */
    CHEMK_CELL_ROUTED_DI = 8  /* info bit (ANN mode): the cell was advanced by DI */
};

/* Largest species count: one wavefront (64 lanes) holds the K+1 unknowns. */
#define CHEMK_MAX_SPECIES 63
#define CHEMK_MAX_REACTIONS 4096
#define CHEMK_MAX_ELEMENTS 8

typedef struct chemk_mech chemk_mech;
typedef struct chemk_ctx chemk_ctx;

/* ---- mechanism ------------------------------------------------------------
 * Reaction j reads  sum_i reactants[2j+i]  (+M)  <=>  sum_i products[2j+i] (+M),
 * slot value -1 = empty, a species may appear in both slots (2A).  Rates are
 * mass action with k_f = A T^beta exp(-Ea/(R_c T)) (cgs, Ea in cal/mol), the
 * reverse rate from the equilibrium constant K_c = K_p (p0/(R_u T))^dnu with
 * p0 = 101325 Pa and K_p from the NASA-7 Gibbs energies, and third bodies with
 * unit efficiencies ([M] = p/(R_u T)) multiplying both directions.  NASA-7 is
 * single range: cp/R = a1 + a2 T + .. + a5 T^4, h/RT = a1 + a2 T/2 + .. + a6/T,
 * s/R = a1 ln T + a2 T + .. + a7.  All arrays are HOST memory, copied.      */
typedef struct {
    int32_t n_elements;           /* E, 1..CHEMK_MAX_ELEMENTS                     */
    int32_t n_species;            /* K, 1..CHEMK_MAX_SPECIES                      */
    int32_t n_reactions;          /* R, 0..CHEMK_MAX_REACTIONS                    */
    const double *element_mass;   /* [E] g/mol, > 0                               */
    const int32_t *composition;   /* [K*E] atoms of element e in species k, >= 0  */
    const double *nasa7;          /* [K*7]                                        */
    const int32_t *reactants;     /* [R*2] species index or -1                    */
    const int32_t *products;      /* [R*2] species index or -1                    */
    const double *log_A;          /* [R] natural log of A, cgs                    */
    const double *beta;           /* [R]                                          */
    const double *Ea;             /* [R] cal/mol                                  */
    const int32_t *third_body;    /* [R] 0/1                                      */
    const int32_t *reversible;    /* [R] 0/1                                      */
} chemk_mech_desc;

/* Validate and copy a mechanism.  Rejects (CHEMK_E_MECH, message in
 * chemk_last_error) reactions that do not conserve every element, empty
 * sides, out-of-range indices, species without atoms and non-finite numbers. */
int chemk_mech_create(const chemk_mech_desc *desc, chemk_mech **out);
void chemk_mech_free(chemk_mech *mech);
int chemk_mech_info(const chemk_mech *mech, int32_t *K, int32_t *R, int32_t *E);

/* A context owns the device copy of one mechanism plus scratch, queues,
 * captured graphs, the autotune cache and the optional network, on `device`.
 * The mechanism may be freed after this call.                               */
int chemk_ctx_create(int device, const chemk_mech *mech, chemk_ctx **out);
void chemk_ctx_free(chemk_ctx *ctx);

/* Message of the last failed call on this thread ("" if none). */
const char *chemk_last_error(void);

/* ---- properties (Sec. II.A: thermal property update) --------------------- */

/* Mixture cp [J/(kg K)] and h [J/kg] of n cells at (T[c], Y[c,:]). */
int chemk_thermo(chemk_ctx *ctx, int64_t n, const double *T, const double *Y,
                 double *cp, double *h, void *stream);

/* T from the mixture enthalpy: Newton on h(T, Y) = h[c] starting from the
 * value in T[c] (relative tolerance 1e-12, at most 50 iterations), then
 * bisection on [200, 4000] K.  T is in/out; status[c] = 0 or
 * CHEMK_CELL_NEWTON (h outside [h(200 K), h(4000 K)]; T left unchanged). */
int chemk_T_from_h(chemk_ctx *ctx, int64_t n, const double *h, const double *Y,
                   double *T, int32_t *status, void *stream);

/* Right-hand side of Eq. 1 at constant p: dydt[c*(K+1) + k] = dY_k/dt for
 * k < K and dT/dt at k = K.                                                  */
int chemk_rhs(chemk_ctx *ctx, int64_t n, const double *T, const double *p,
              const double *Y, double *dydt, void *stream);

/* Analytic Jacobian of chemk_rhs w.r.t. (Y_1..Y_K, T), row-major (K+1)^2 per
 * cell: J[c*(K+1)^2 + i*(K+1) + j] = d f_i / d y_j.                          */
int chemk_jacobian(chemk_ctx *ctx, int64_t n, const double *T, const double *p,
                   const double *Y, double *J, void *stream);

/* ---- the steps either side of the advance ------------------------------------ */
/* Transport properties (Sec. II.A: properties updated from temperature
 * polynomials).  chemk_transport_set stores, per species k, the coefficients
 * of ln mu_k [Pa s] and ln lambda_k [W/(m K)] as cubic polynomials in ln T
 * (ascending powers; mu_poly, lam_poly host arrays [K*4]).  chemk_transport
 * then gives per cell the mixture viscosity by Wilke's rule,
 *   mu = sum_i X_i mu_i / sum_j X_j (1 + (mu_i/mu_j)^(1/2) (W_j/W_i)^(1/4))^2
 *        / (8 (1 + W_i/W_j))^(1/2),
 * and the conductivity by the average of Mathur, Tondon and Saxena,
 *   lambda = (sum_k X_k lambda_k + 1 / sum_k X_k / lambda_k) / 2,
 * X the mole fractions of Y.  T [n], Y [n, K] in; mu [n] and lam [n] (NULL
 * allowed) out; device arrays, asynchronous on `stream`.  CHEMK_E_STATE
 * before chemk_transport_set.                                               */
int chemk_transport_set(chemk_ctx *ctx, const double *mu_poly, const double *lam_poly);
int chemk_transport(chemk_ctx *ctx, int64_t n, const double *T, const double *Y, double *mu,
                    double *lam, void *stream);

/* The PaSR closure of one flow step (Sec. III: the network or DI replaces
 * only the integration inside the partially stirred reactor model).  From the
 * state before (T, p, Y0) and after (Y1) the chemistry advance over dt, per
 * cell: rho the density of (T, p, Y0); omega_k = rho (Y1_k - Y0_k) / dt;
 * tau_c = max over species with omega_k > 0 and Y1_k >= y_min of
 * rho Y1_k / omega_k (the slowest formation; none: kappa = 1);
 * u' = (2 k_sgs / 3)^(1/2), tau_Delta = delta / u',
 * epsilon = c_eps k_sgs^(3/2) / delta, tau_K = (mu / rho / epsilon)^(1/2),
 * tau_mix = (tau_Delta tau_K)^(1/2) (k_sgs <= 0: kappa = 0);
 * kappa = tau_c / (tau_c + tau_mix).  Outputs (NULL allowed, not all):
 * kappa [n], omega [n, K] = kappa omega_k in kg/(m^3 s), Y_out [n, K] =
 * Y0 + kappa (Y1 - Y0).  k_sgs [m^2/s^2], delta [m] (filter width) and mu
 * [Pa s] (e.g. from chemk_transport) are per cell.  Defaults of the
 * readings: c_eps = 1.048, y_min = 1e-6.  Device arrays, asynchronous.      */
int chemk_pasr(chemk_ctx *ctx, int64_t n, const double *T, const double *p, const double *Y0,
               const double *Y1, double dt, const double *k_sgs, const double *delta,
               const double *mu, double c_eps, double y_min, double *kappa, double *omega,
               double *Y_out, void *stream);

/* ---- the chemistry advance (Eqs. 1-2) --------------------------------------- */
enum { CHEMK_MODE_DI = 0, CHEMK_MODE_ANN = 1 };

typedef struct {
    int32_t mode;            /* CHEMK_MODE_DI or CHEMK_MODE_ANN                    */
    int32_t max_steps;       /* DI step limit per cell (default 100000)            */
    double rtol;             /* DI relative tolerance (default 1e-7)               */
    double atol_Y;           /* DI absolute tolerance on Y (default 1e-14)         */
    double atol_T;           /* DI absolute tolerance on T [K] (default 1e-6)      */
    double h0_frac;          /* first trial step = h0_frac * dt (default 1e-3)     */
    int32_t bins;            /* stiffness bins; 0 = autotuned / cached choice      */
    int32_t waves_per_cu;    /* persistent DI residency; 0 = autotuned / default   */
    int32_t use_graph;       /* 1 = capture the whole step in a hipGraph and replay */
    int32_t project;         /* 1 = FP64 element projection of the output (default) */
    int32_t di_kernel;       /* DI factorisation: CHEMK_DI_AUTO (default), CHEMK_DI_LDS_LU or
                                CHEMK_DI_REG_LU; both give the same numbers            */
} chemk_opts;

/* DI kernel variants.  The LDS LU keeps the iteration matrix in the wave's
 * LDS slice and handles any N = K + 1 <= 64; the register LU keeps each row in
 * registers and exists for N = 10 and 33 (CHEMK_DI_REG_LU on another N is
 * CHEMK_E_ARG).  CHEMK_DI_AUTO takes the register LU where it exists.       */
enum { CHEMK_DI_AUTO = 0, CHEMK_DI_LDS_LU = 1, CHEMK_DI_REG_LU = 2 };

void chemk_opts_default(chemk_opts *opts);

/* Advance n cells over dt in place.  T [n] and Y [n,K] are in/out, p [n] in.
 * DI: adaptive Rosenbrock (RODAS, order 4(3)) on y = (Y, T); the final T is
 * recovered from the conserved mixture enthalpy and Y is projected so that
 * element masses equal the input's to FP64 round-off.
 * ANN: the trained network predicts Y(t+dt) - Y(t); the prediction is
 * element-projected; cells outside the training envelope or whose prediction
 * fails the checks (non-finite, Y_k below -neg_tol) are advanced by DI in the
 * same call and get CHEMK_CELL_ROUTED_DI set in status.  dt must equal the
 * trained dt (relative 1e-12) else CHEMK_E_DT and nothing is touched.
 * status [n] (required) receives the per-cell code; nsteps [n] (optional,
 * NULL allowed) receives the accepted+rejected DI step count (0 for ANN).   */
int chemk_advance(chemk_ctx *ctx, int64_t n, double *T, const double *p, double *Y,
                  double dt, const chemk_opts *opts, int32_t *status, int32_t *nsteps,
                  void *stream);

/* The advance for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * chemk_advance in DI mode, with the step's stiffness bins, queue and
 * counters in a fixed device array of the library instead of the context's
 * buffers.  The array (about 2 MiB) exists once per GPU and is held until the
 * process ends; its address is looked up when a context is created.  The call
 * allocates nothing: no hipMalloc/hipFree, no graph, no timing events
 * (use_graph and phase timing are ignored; the step is enqueued eagerly).
 * opts->mode must be CHEMK_MODE_DI and n at most CHEMK_NOALLOC_MAX_CELLS,
 * else CHEMK_E_ARG.  Results equal chemk_advance's.  Every call on one GPU,
 * from any context or thread, shares that GPU's array, which keeps the last
 * call's contents: calls that overlap on one GPU (other streams, threads)
 * race, so the caller serialises them.  chemk_last_counters then reports this
 * call's counters.                                                         */
#define CHEMK_NOALLOC_MAX_CELLS 262144
int chemk_advance_noalloc(chemk_ctx *ctx, int64_t n, double *T, const double *p, double *Y,
                          double dt, const chemk_opts *opts, int32_t *status, int32_t *nsteps,
                          void *stream);

/* Stiffness-batching autotuner (the "bins / tile shape" choice of the DI
 * path): runs DI on COPIES of the n given cells for a small grid of
 * (stiffness bins, persistent waves per CU), then, where the register LU
 * exists, the LDS LU at the best pair; times each with HIP events on
 * `stream`, stores the fastest in the context (used whenever opts->bins,
 * opts->waves_per_cu or opts->di_kernel is 0) and returns it in
 * best[0] = bins, best[1] = waves_per_cu, best_ms[0] = its time.
 * Results are cached for the process, keyed by (GPU architecture, compute
 * units, K, R, E, floor(log2 n)): a later call with the same key takes the
 * cached choice without running anything (best_ms = the time measured
 * then).  With the environment variable CHEMK_TUNE_CACHE naming a file, the
 * cache is read from it on first use and rewritten after each new entry
 * (one entry per line).  Synchronises `stream` when it tunes.  The state
 * arrays are not modified.                                                  */
int chemk_autotune(chemk_ctx *ctx, int64_t n, const double *T, const double *p,
                   const double *Y, double dt, const chemk_opts *opts, int32_t best[2],
                   double *best_ms, void *stream);

/* The context's tuned choice: out[0] = bins, out[1] = waves per CU,
 * out[2] = DI factorisation (CHEMK_DI_*); zeros before any tuning.          */
int chemk_tuning(chemk_ctx *ctx, int32_t out[3]);

/* Empties the process's autotuner cache (not the CHEMK_TUNE_CACHE file).    */
void chemk_tune_cache_clear(void);

/* Phase timing (profiling aid).  While enabled, chemk_advance runs eagerly
 * (use_graph is ignored) and brackets each phase's launches with HIP events
 * on the caller's stream (chemk_ann_forward_packed brackets its layer
 * launches too); chemk_timing_read synchronises the stream and
 * returns, per phase, the summed milliseconds and the number of launches
 * since the last read (then resets).  Phases: */
enum {
    CHEMK_PHASE_DI = 0,        /* persistent DI kernel (DI mode)                  */
    CHEMK_PHASE_BINNING = 1,   /* stiffness key, histogram, queue                  */
    CHEMK_PHASE_INGEST = 2,    /* ANN: features, envelope test                     */
    CHEMK_PHASE_MLP = 3,       /* ANN: the MLP GEMMs                               */
    CHEMK_PHASE_POST = 4,      /* ANN: de-normalise, project, check, T             */
    CHEMK_PHASE_FALLBACK = 5,  /* ANN: DI on the routed cells                      */
    CHEMK_PHASE_LAYER1 = 6,    /* ANN: the GEMM launches of layer 1, 2, 3 and of   */
    CHEMK_PHASE_LAYER2 = 7,    /*      layer 4 and beyond, each also counted in    */
    CHEMK_PHASE_LAYER3 = 8,    /*      CHEMK_PHASE_MLP                             */
    CHEMK_PHASE_LAYER4 = 9,
    CHEMK_NUM_PHASES = 10
};
int chemk_timing(chemk_ctx *ctx, int32_t enable);
int chemk_timing_read(chemk_ctx *ctx, double ms[CHEMK_NUM_PHASES],
                      int64_t launches[CHEMK_NUM_PHASES], void *stream);

/* Counters of the last chemk_advance on this context (synchronises stream):
 * out[0] cells routed to DI, out[1] total DI steps, out[2] cells with a
 * non-zero status (ignoring the routed bit).                                 */
int chemk_last_counters(chemk_ctx *ctx, int64_t out[3], void *stream);

/* ---- the learned part (Sec. II.B) ------------------------------------------
 * One MLP: dims[0] = K + 2 inputs (Box-Cox(max(Y,0)) with lambda = 0.1, T, p,
 * each z-scored), hidden dims[1..L-1] with GELU, dims[L] = K outputs (the
 * z-scored change of Y over dt).  BF16 operands on MFMA with FP32
 * accumulation; FP32 master weights for training.  Parameter vector layout
 * (host, FP32): for each layer l: W_l [dims[l] x dims[l+1]] row-major, then
 * b_l [dims[l+1]].                                                           */
int chemk_ann_create(chemk_ctx *ctx, const int32_t *dims, int32_t n_layers);

/* One network per species (Sec. II.B: training and prediction are done for
 * each species' mass fraction separately): K MLPs of the same shape, dims[0] =
 * K + 2, hidden dims[1..L-1] (n_layers >= 2), dims[L] = 1, network k
 * predicting the z-scored change of Y_k.  Replaces the context's network like
 * chemk_ann_create and serves chemk_advance and chemk_ann_forward_packed as a
 * K-output network would.  Parameter vector: the K networks' vectors (each in
 * the layout above with dims[L] = 1) one after the other, species order.  The
 * K networks run as one product for the first layer, one grouped product per
 * hidden layer, and the output layer fused into the last hidden layer (one
 * block-diagonal product with one hidden layer).  Trainable in place:
 * chemk_ann_train_step and chemk_ann_train then take one step of all K
 * networks at once (grouped products), network k's loss the mean squared
 * error of its own output column of Z (Eq. 8 for one species); the batch
 * loss reported is the mean over the networks.  The physics losses and
 * out_w couple the species and are refused (CHEMK_E_UNSUPPORTED).  A network
 * can also be trained alone as a K-output network with a one-hot out_w and
 * its output row k kept.                                                     */
int chemk_ann_create_species(chemk_ctx *ctx, const int32_t *dims, int32_t n_layers);
int chemk_ann_param_count(chemk_ctx *ctx, int64_t *count);
int chemk_ann_set_weights(chemk_ctx *ctx, const float *params, int64_t count);
int chemk_ann_get_weights(chemk_ctx *ctx, float *params, int64_t count);

/* Normalisation (host arrays): mu_x/sd_x [K+2] over raw features, mu_y/sd_y
 * [K] over Y(t+dt)-Y(t); dt is the step the network is trained for.          */
int chemk_ann_set_norm(chemk_ctx *ctx, const double *mu_x, const double *sd_x,
                       const double *mu_y, const double *sd_y, double dt);
int chemk_ann_get_norm(chemk_ctx *ctx, double *mu_x, double *sd_x, double *mu_y,
                       double *sd_y, double *dt);

/* Training envelope (host arrays): raw-feature box lo/hi [K+2]; a cell with
 * any feature outside it is routed to DI.  neg_tol: predicted Y_k below
 * -neg_tol routes the cell to DI.                                            */
int chemk_ann_set_envelope(chemk_ctx *ctx, const double *lo, const double *hi, double neg_tol);
int chemk_ann_get_envelope(chemk_ctx *ctx, double *lo, double *hi, double *neg_tol);

/* Checks that decide, per cell, whether the network's step is kept or the cell
 * is advanced by DI in the same call (ANN mode).
 *
 * Input side (ingest), besides the raw-feature box above: up to
 * CHEMK_MAX_RATIOS element-ratio windows, after the paper's filters on its
 * training states (windows on the molar H/C and O/N ratios and on the
 * equivalence ratio, Sec. II.B).  With z_e = sum_k Y_k n_ek A_e / W_k the mass
 * fraction of element e (elements in the mechanism's order), window j accepts
 * a cell when
 *     ratio_lo[j] <= (sum_e ratio_num[j*8+e] z_e) / (sum_e ratio_den[j*8+e] z_e)
 *                 <= ratio_hi[j]
 * and the denominator is positive (a molar ratio n_a / n_b has num = 1/A_a at
 * a and den = 1/A_b at b).
 *
 * Output side (post step): a cell is routed when the element-conserving
 * correction of the prediction moves some species by more than adj_max times
 * its training spread sd_y[k] (adj_max <= 0: no limit), or when
 * T(t+dt) - T(t) falls outside [dT_lo, dT_hi] K.  chemk_ann_create sets every
 * check off (no windows, no limit, dT window of +-1e300).                   */
#define CHEMK_MAX_RATIOS 4
typedef struct {
    double adj_max;
    double dT_lo, dT_hi;
    int32_t n_ratios;                                           /* 0..CHEMK_MAX_RATIOS */
    double ratio_num[CHEMK_MAX_RATIOS * CHEMK_MAX_ELEMENTS];    /* [j*8 + e]           */
    double ratio_den[CHEMK_MAX_RATIOS * CHEMK_MAX_ELEMENTS];
    double ratio_lo[CHEMK_MAX_RATIOS], ratio_hi[CHEMK_MAX_RATIOS];
} chemk_ann_checks;
int chemk_ann_set_checks(chemk_ctx *ctx, const chemk_ann_checks *checks);
int chemk_ann_get_checks(chemk_ctx *ctx, chemk_ann_checks *checks);

/* Device: fit the input envelope and the dT window to n training states.
 * For each raw feature (K + 2), each element-ratio window already set
 * (n_ratios and its coefficients; its value taken over the states with a
 * positive denominator) and, when T_next [n] is given, for T_next - T: the q
 * and 1 - q quantiles, widened by widen times their distance on each side,
 * become the feature's [lo, hi] (box, ratio window or dT window); the lower
 * bound of each mass-fraction feature is extended down to Box-Cox(0) = -10,
 * so that a species absent from a cell never routes it.  Quantiles
 * are resolved on 4096 bins over each value's full range and rounded outwards
 * to bin edges, so q = 0 gives the exact minimum and maximum.  Requires
 * 0 <= q < 0.5, widen >= 0, n >= 2.  Synchronises `stream`.                 */
int chemk_ann_fit_envelope(chemk_ctx *ctx, int64_t n, const double *T, const double *p,
                           const double *Y, const double *T_next, double q, double widen,
                           void *stream);

/* Device: compute the normalisation from n training pairs (state, state after
 * dt) and store it (sd floored at 1e-12), plus the envelope box of the raw
 * features widened by `widen` times its span on each side.                   */
int chemk_ann_fit_norm(chemk_ctx *ctx, int64_t n, const double *T, const double *p,
                       const double *Y, const double *Y_next, double dt, double widen,
                       double neg_tol, void *stream);

/* Device: pack training pairs into network space: X [n, 64] BF16 (the
 * dims[0] = K + 2 features zero padded to 64 columns, stored as uint16 bit
 * patterns; X 16-byte aligned, else CHEMK_E_ARG) and, when Y_next is given,
 * the z-scored targets Z [n, K] FP32.                                         */
int chemk_ann_pack(chemk_ctx *ctx, int64_t n, const double *T, const double *p,
                   const double *Y, const double *Y_next, uint16_t *X, float *Z,
                   void *stream);

/* Network forward on packed inputs X [n, 64] (BF16 bits): out [n, K] FP32, the
 * z-scored prediction.  Test hook and batch inference.                        */
int chemk_ann_forward_packed(chemk_ctx *ctx, int64_t n, const uint16_t *X, float *out,
                             void *stream);

/* Per-row weights of the heat-release loss (Sec. II.B, Eq. 10) for n
 * training pairs: HRR = -(rho / dt) sum_k h_k(T) dY_k [W/m^3] over the step,
 * h_k the species enthalpy per unit mass at the input T (NASA-7), rho the
 * input density.  With sigma_k the stored sd of dY (chemk_ann_set_norm) and
 * s the scale, G [n, K] FP32 (device) receives
 *     G_ik = -(rho_i / dt) h_k(T_i) sigma_k / s,
 * so that sum_k G_ik (out_ik - z_ik) = (HRR*_i - HRR_i) / s for the network's
 * z-scored prediction out and target z.  scale_in > 0 fixes s (the training
 * set's, for a held-out set); scale_in = 0 takes s = RMS of the DI label
 * HRR_i over the n rows (Y_next - Y the label).  *scale_out (host, may be
 * NULL) receives s.  Synchronises `stream`.                                  */
int chemk_ann_hrr_weights(chemk_ctx *ctx, int64_t n, const double *T, const double *p,
                          const double *Y, const double *Y_next, double dt, double scale_in,
                          float *G, double *scale_out, void *stream);

/* One training step on rows idx[0..B-1] of (X, Z): forward with saved
 * activations, the loss, backward, Adam (beta1 0.9, beta2 0.999, eps 1e-8,
 * step counter kept in the context) with learning rate lr.  The loss is
 * Eq. 11 with W1 = 1 on the z-scored outputs out (Eq. 8: mean of
 * (out - z)^2 over the B K values) plus
 *   w_mass * mean_i |sum_k (mu_k + sigma_k out_ik)| / sum_k sigma_k
 *     (Eq. 9: the predicted Y(t+dt) sums to one plus sum_k dY*_k, the
 *     inputs summing to one; scaled by the spread of dY),
 *   w_hrr * mean_i (sum_k G_ik (out_ik - z_ik))^2
 *     (Eq. 10 in units of the scale of chemk_ann_hrr_weights),
 * with G [rows of X, K] the weights of chemk_ann_hrr_weights (NULL allowed
 * when w_hrr = 0).  out_w (device FP32 [K], may be NULL) weights the data
 * term per output: sum_k w_k (out_ik - z_ik)^2 / (B sum_k w_k) replaces the
 * plain mean (all w_k = 1 when NULL); a one-hot out_w trains a network on one
 * species alone (the per-species ensemble the paper names as an alternative
 * in Sec. II.B).  Weights must be finite, >= 0 and not all zero, else
 * CHEMK_E_ARG.  loss (device FP32 scalar, may
 * be NULL) receives the batch loss before the update.  grads (device FP32
 * [param_count], may be NULL) receives the gradient in the layout of
 * chemk_ann_get_weights; with update = 0 the weights are left unchanged.      */
int chemk_ann_train_step(chemk_ctx *ctx, const int32_t *idx, int32_t B, const uint16_t *X,
                         const float *Z, const float *G, float w_mass, float w_hrr,
                         const float *out_w, float lr, int32_t update, float *loss,
                         float *grads, void *stream);

/* The training loop (Sec. II.B: Adam on the loss of Eq. 8), on the device.
 * Rows of the packed training set (X [n, 64] BF16 bits, 16-byte aligned; Z
 * [n, K] FP32 z-scored targets, as written by chemk_ann_pack) are visited in
 * a new pseudo-random order each epoch: row r of batch b of epoch e is
 * perm_e(b * batch + r), perm_e a four-round Feistel permutation of [0, n)
 * (cycle walking; round function SplitMix64's mixer) keyed by `seed` and e,
 * so each epoch takes floor(n / batch) batches of distinct rows.  Each step is
 * chemk_ann_train_step (with opts' loss weights and G) with the learning
 * rate of a cosine schedule from lr0 to lr1 over all steps, lr1 + (lr0 - lr1)(1 + cos(pi s / S)) / 2 at step s
 * of S; the Adam step count continues from the context's.  With use_graph = 1
 * one step is captured in a hipGraph and replayed.  After each epoch the mean
 * squared error (the data loss alone) over the n_hold held-out rows (X_hold, Z_hold; n_hold = 0
 * skips it) is evaluated.  epoch_loss and hold_loss (HOST arrays [epochs],
 * NULL allowed) receive the epoch's mean batch loss and the held-out loss.
 * Synchronises `stream`.                                                    */
typedef struct {
    int32_t batch;           /* rows per step: a multiple of 64, <= n           */
    int32_t epochs;
    float lr0, lr1;          /* cosine learning-rate schedule, first -> last     */
    uint64_t seed;           /* key of the per-epoch permutations                 */
    int32_t use_graph;       /* 1 = replay one captured training step            */
    float w_mass, w_hrr;     /* weights of the mass and heat-release losses (W2, W3
                                of Eq. 11, chemk_ann_train_step); 0 = data loss only */
    const float *G;          /* [n, K] heat-release weights (w_hrr > 0), device  */
    const float *out_w;      /* [K] per-output weights of the data term
                                (chemk_ann_train_step), device; NULL = all 1     */
    int32_t epoch0;          /* this call runs epochs [epoch0, epoch0 + epochs)   */
    int32_t epochs_total;    /* of a schedule over this many epochs (0: epoch0 +
                                epochs): the learning rate, the row orders and
                                the Adam step count continue as if one call ran
                                them all; epoch_loss / hold_loss get this call's
                                epochs                                           */
} chemk_train_opts;
int chemk_ann_train(chemk_ctx *ctx, int64_t n, const uint16_t *X, const float *Z,
                    const uint16_t *X_hold, const float *Z_hold, int64_t n_hold,
                    const chemk_train_opts *opts, float *epoch_loss, float *hold_loss,
                    void *stream);

/* Reset the Adam moments and step counter. */
int chemk_ann_reset_optimizer(chemk_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* CHEMK_H */
