// api.cpp -- the C ABI: argument validation, mechanism tables, contexts, the
// DI/ANN step sequencing, graph capture and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "chemk.h"
#include "chemk_dev.h"
#include "chemk_internal.h"
#include "ann_internal.h"

using namespace chemk;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(CHEMK_E_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                        __FILE__, __LINE__);                                            \
    } while (0)

extern "C" const char *chemk_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// mechanism (host copy)
// ---------------------------------------------------------------------------
struct chemk_mech {
    int E = 0, K = 0, R = 0;
    std::vector<double> emass, nasa, lnA, beta, Ea;
    std::vector<int> comp, reac, prod, tb, rev;
};

extern "C" int chemk_mech_create(const chemk_mech_desc *d, chemk_mech **out) {
    g_err.clear();
    if (!d || !out) return fail(CHEMK_E_ARG, "null descriptor or output pointer");
    *out = nullptr;
    const int E = d->n_elements, K = d->n_species, R = d->n_reactions;
    if (E < 1 || E > CHEMK_MAX_ELEMENTS)
        return fail(CHEMK_E_MECH, "n_elements=%d outside [1, %d]", E, CHEMK_MAX_ELEMENTS);
    if (K < 1 || K > CHEMK_MAX_SPECIES)
        return fail(CHEMK_E_MECH, "n_species=%d outside [1, %d]", K, CHEMK_MAX_SPECIES);
    if (R < 0 || R > CHEMK_MAX_REACTIONS)
        return fail(CHEMK_E_MECH, "n_reactions=%d outside [0, %d]", R, CHEMK_MAX_REACTIONS);
    if (!d->element_mass || !d->composition || !d->nasa7)
        return fail(CHEMK_E_ARG, "null element_mass / composition / nasa7");
    if (R > 0 && (!d->reactants || !d->products || !d->log_A || !d->beta || !d->Ea ||
                  !d->third_body || !d->reversible))
        return fail(CHEMK_E_ARG, "null reaction array");
    auto m = std::make_unique<chemk_mech>();
    m->E = E;
    m->K = K;
    m->R = R;
    m->emass.assign(d->element_mass, d->element_mass + E);
    m->comp.assign(d->composition, d->composition + (size_t)K * E);
    m->nasa.assign(d->nasa7, d->nasa7 + (size_t)K * 7);
    for (int e = 0; e < E; ++e)
        if (!(std::isfinite(m->emass[e]) && m->emass[e] > 0))
            return fail(CHEMK_E_MECH, "element %d: mass must be finite and > 0", e);
    for (int k = 0; k < K; ++k) {
        int atoms = 0;
        for (int e = 0; e < E; ++e) {
            if (m->comp[k * E + e] < 0)
                return fail(CHEMK_E_MECH, "species %d: negative atom count", k);
            atoms += m->comp[k * E + e];
        }
        if (atoms == 0) return fail(CHEMK_E_MECH, "species %d has no atoms", k);
        for (int j = 0; j < 7; ++j)
            if (!std::isfinite(m->nasa[k * 7 + j]))
                return fail(CHEMK_E_MECH, "species %d: non-finite NASA-7 coefficient", k);
    }
    if (R > 0) {
        m->reac.assign(d->reactants, d->reactants + 2 * R);
        m->prod.assign(d->products, d->products + 2 * R);
        m->lnA.assign(d->log_A, d->log_A + R);
        m->beta.assign(d->beta, d->beta + R);
        m->Ea.assign(d->Ea, d->Ea + R);
        m->tb.assign(d->third_body, d->third_body + R);
        m->rev.assign(d->reversible, d->reversible + R);
    }
    for (int j = 0; j < R; ++j) {
        int nr = 0, np = 0;
        std::vector<long> bal(E, 0);
        for (int i = 0; i < 2; ++i) {
            const int a = m->reac[2 * j + i], b = m->prod[2 * j + i];
            if (a < -1 || a >= K || b < -1 || b >= K)
                return fail(CHEMK_E_MECH, "reaction %d: species index out of range", j);
            if (a >= 0) {
                ++nr;
                for (int e = 0; e < E; ++e) bal[e] -= m->comp[a * E + e];
            }
            if (b >= 0) {
                ++np;
                for (int e = 0; e < E; ++e) bal[e] += m->comp[b * E + e];
            }
        }
        if (m->reac[2 * j] < 0 || m->prod[2 * j] < 0)
            return fail(CHEMK_E_MECH, "reaction %d: slot 0 of each side must be filled", j);
        (void)nr;
        (void)np;
        for (int e = 0; e < E; ++e)
            if (bal[e] != 0)
                return fail(CHEMK_E_MECH, "reaction %d does not conserve element %d", j, e);
        if (!std::isfinite(m->lnA[j]) || !std::isfinite(m->beta[j]) || !std::isfinite(m->Ea[j]))
            return fail(CHEMK_E_MECH, "reaction %d: non-finite Arrhenius parameter", j);
        if ((m->tb[j] != 0 && m->tb[j] != 1) || (m->rev[j] != 0 && m->rev[j] != 1))
            return fail(CHEMK_E_MECH, "reaction %d: flags must be 0 or 1", j);
    }
    *out = m.release();
    return CHEMK_OK;
}

extern "C" void chemk_mech_free(chemk_mech *m) { delete m; }

extern "C" int chemk_mech_info(const chemk_mech *m, int32_t *K, int32_t *R, int32_t *E) {
    if (!m) return fail(CHEMK_E_ARG, "null mechanism");
    if (K) *K = m->K;
    if (R) *R = m->R;
    if (E) *E = m->E;
    return CHEMK_OK;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
// A captured step is replayed only for the same arguments and, in ANN mode,
// the same generation of the network's state (buffers, tables and checks
// that the graph holds by address or by value).
struct GraphKey {
    int64_t n;
    const void *T, *p, *Y, *st, *ns;
    double dt;
    int mode, bins, wpc, max_steps, project;
    double rtol, atolY, atolT, h0;
    uint64_t ann_gen;
    bool operator<(const GraphKey &o) const {
        return std::tie(n, T, p, Y, st, ns, dt, mode, bins, wpc, max_steps, project, rtol, atolY,
                        atolT, h0, ann_gen) < std::tie(o.n, o.T, o.p, o.Y, o.st, o.ns, o.dt, o.mode,
                                                       o.bins, o.wpc, o.max_steps, o.project, o.rtol,
                                                       o.atolY, o.atolT, o.h0, o.ann_gen);
    }
};

struct chemk_ctx {
    int device = 0;
    int cu_count = 256;
    int K = 0, R = 0, E = 0, N = 0;
    DevMech dm{};
    void *tables = nullptr;
    // DI scratch, grown on demand
    int64_t cap = 0;
    int *bin = nullptr, *queue = nullptr;
    int *small = nullptr;                 // [0] counter, [1] n_items, [2..] hist/offs
    unsigned long long *stats = nullptr;  // [0] routed, [1] steps, [2] failed
    unsigned long long *last_stats = nullptr;   // where the last advance wrote its counters
    void *noalloc = nullptr;              // this device's copy of the no-allocation scratch
    int tuned_bins = 0, tuned_wpc = 0, tuned_variant = 0;
    std::string arch;                     // gcnArchName of the device
    std::map<GraphKey, hipGraphExec_t> graphs;
    AnnState *ann = nullptr;
    void *transport = nullptr;            // transport-property tables (closure.hip)
    PhaseTimer timer;
};

static constexpr int kMaxBins = 256;

// accessors for the learned part (ann.hip)
AnnState *&ctx_ann(chemk_ctx *c) { return c->ann; }
void *&ctx_transport(chemk_ctx *c) { return c->transport; }
chemk::PhaseTimer *ctx_timer(chemk_ctx *c) { return c->timer.on ? &c->timer : nullptr; }
int ctx_device(chemk_ctx *c) { return c->device; }
int ctx_K(chemk_ctx *c) { return c->K; }
void ctx_set_error(const char *msg) { g_err = msg; }
chemk::DevMech ctx_devmech(chemk_ctx *c) { return c->dm; }

static int set_device(chemk_ctx *c) {
    HIP_TRY(hipSetDevice(c->device));
    return CHEMK_OK;
}

// ---------------------------------------------------------------------------
// the DI advance without allocation: its scratch in a static device array
// ---------------------------------------------------------------------------
// Layout (bytes): statistics [4 u64] at 0, counters/histogram/offsets
// [2 + 2 kMaxBins int] at kNaSmall, bins and queue [CHEMK_NOALLOC_MAX_CELLS
// int each] after them.  Every GPU holds its own copy until the process ends.
constexpr size_t kNaSmall = 256;
constexpr size_t kNaBin = kNaSmall + ((sizeof(int) * (2 + 2 * kMaxBins) + 255) & ~size_t(255));
constexpr size_t kNaQueue = kNaBin + sizeof(int) * CHEMK_NOALLOC_MAX_CELLS;
constexpr size_t kNaBytes = kNaQueue + sizeof(int) * CHEMK_NOALLOC_MAX_CELLS;
static __device__ __align__(256) unsigned char scratch[kNaBytes];

// The device address of this GPU's `scratch`, looked up once per device with
// that device current (the array's name in host code is not a device address).
static int noalloc_address(int device, void **out) {
    static std::mutex mu;
    static void *addr[64] = {};
    if (device < 0 || device >= 64) return fail(CHEMK_E_UNSUPPORTED, "device %d >= 64", device);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(CHEMK_E_HIP, "hipGetSymbolAddress returned a null address");
        addr[device] = ptr;
    }
    *out = addr[device];
    return CHEMK_OK;
}


extern "C" int chemk_ctx_create(int device, const chemk_mech *m, chemk_ctx **out) {
    g_err.clear();
    if (!m || !out) return fail(CHEMK_E_ARG, "null mechanism or output pointer");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return fail(CHEMK_E_ARG, "device %d outside [0, %d)", device, ndev);
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(CHEMK_E_UNSUPPORTED, "device %d is %s; this library is built for gfx950",
                    device, prop.gcnArchName);
    auto c = std::make_unique<chemk_ctx>();
    c->device = device;
    c->cu_count = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    c->K = m->K;
    c->R = m->R;
    c->E = m->E;
    c->N = m->K + 1;
    const int K = m->K, R = m->R, E = m->E;
    if (di_template_N(c->N) < 0) return fail(CHEMK_E_UNSUPPORTED, "K=%d too large", K);
    if (di_block_lds_bytes(K, R) > 64 * 1024)
        return fail(CHEMK_E_UNSUPPORTED, "mechanism needs %zu bytes of LDS per DI workgroup (> 64 KiB)",
                    di_block_lds_bytes(K, R));

    // host-side tables
    std::vector<double> W(K), invW(K);
    for (int k = 0; k < K; ++k) {
        double w = 0;
        for (int e = 0; e < E; ++e) w += m->comp[k * E + e] * m->emass[e];
        W[k] = w;
        invW[k] = 1.0 / w;
    }
    std::vector<int4> rsp(std::max(R, 1));
    std::vector<double4> rpar(std::max(R, 1));
    std::vector<int4> rflag(std::max(R, 1));
    std::vector<std::vector<std::pair<int, double>>> inc(K);
    for (int j = 0; j < R; ++j) {
        int a0 = m->reac[2 * j], a1 = m->reac[2 * j + 1], p0 = m->prod[2 * j],
            p1 = m->prod[2 * j + 1];
        // keep filled slots first
        if (a0 < 0) std::swap(a0, a1);
        if (p0 < 0) std::swap(p0, p1);
        rsp[j] = make_int4(a0, a1, p0, p1);
        const int nf = (a0 >= 0) + (a1 >= 0), nr = (p0 >= 0) + (p1 >= 0);
        rpar[j] = make_double4(m->lnA[j], m->beta[j], m->Ea[j] / RC_CAL, 0.0);
        rflag[j] = make_int4(m->tb[j], m->rev[j], nr - nf, nf + 16 * nr);
        std::map<int, double> nu;
        if (a0 >= 0) nu[a0] -= 1;
        if (a1 >= 0) nu[a1] -= 1;
        if (p0 >= 0) nu[p0] += 1;
        if (p1 >= 0) nu[p1] += 1;
        for (auto &kv : nu)
            if (kv.second != 0.0) inc[kv.first].push_back({j, kv.second});
    }
    std::vector<int> inc_start(K + 1, 0), inc_r;
    std::vector<double> inc_nu;
    for (int k = 0; k < K; ++k) {
        inc_start[k + 1] = inc_start[k] + (int)inc[k].size();
        for (auto &pr : inc[k]) {
            inc_r.push_back(pr.first);
            inc_nu.push_back(pr.second);
        }
    }
    if (inc_r.empty()) {
        inc_r.push_back(0);
        inc_nu.push_back(0.0);
    }
    std::vector<double> Emat((size_t)E * K);
    for (int e = 0; e < E; ++e)
        for (int k = 0; k < K; ++k) Emat[e * K + k] = m->comp[k * E + e] * m->emass[e] / W[k];

    // one device allocation, 256-byte aligned pieces
    struct Piece {
        const void *src;
        size_t bytes;
        size_t off;
    };
    std::vector<Piece> pcs = {
        {W.data(), W.size() * 8, 0},
        {invW.data(), invW.size() * 8, 0},
        {m->nasa.data(), m->nasa.size() * 8, 0},
        {rsp.data(), rsp.size() * sizeof(int4), 0},
        {rpar.data(), rpar.size() * sizeof(double4), 0},
        {rflag.data(), rflag.size() * sizeof(int4), 0},
        {inc_start.data(), inc_start.size() * 4, 0},
        {inc_r.data(), inc_r.size() * 4, 0},
        {inc_nu.data(), inc_nu.size() * 8, 0},
        {Emat.data(), Emat.size() * 8, 0}};
    size_t tot = 0;
    for (auto &pc : pcs) {
        pc.off = tot;
        tot += (pc.bytes + 255) & ~size_t(255);
    }
    std::vector<char> host(tot, 0);
    for (auto &pc : pcs) std::memcpy(host.data() + pc.off, pc.src, pc.bytes);
    if (hipMalloc(&c->tables, tot) != hipSuccess)
        return fail(CHEMK_E_OOM, "hipMalloc(%zu) for mechanism tables failed", tot);
    HIP_TRY(hipMemcpy(c->tables, host.data(), tot, hipMemcpyHostToDevice));
    char *b = (char *)c->tables;
    DevMech &dm = c->dm;
    dm.K = K;
    dm.R = R;
    dm.E = E;
    dm.N = K + 1;
    dm.W = (const double *)(b + pcs[0].off);
    dm.invW = (const double *)(b + pcs[1].off);
    dm.nasa = (const double *)(b + pcs[2].off);
    dm.rsp = (const int4 *)(b + pcs[3].off);
    dm.rpar = (const double4 *)(b + pcs[4].off);
    dm.rflag = (const int4 *)(b + pcs[5].off);
    dm.inc_start = (const int *)(b + pcs[6].off);
    dm.inc_r = (const int *)(b + pcs[7].off);
    dm.inc_nu = (const double *)(b + pcs[8].off);
    dm.Emat = (const double *)(b + pcs[9].off);

    if (int r = noalloc_address(device, &c->noalloc)) return r;
    if (hipMalloc(&c->small, sizeof(int) * (2 + 2 * kMaxBins)) != hipSuccess ||
        hipMalloc(&c->stats, sizeof(unsigned long long) * 4) != hipSuccess)
        return fail(CHEMK_E_OOM, "hipMalloc of context counters failed");
    HIP_TRY(hipMemset(c->stats, 0, sizeof(unsigned long long) * 4));
    *out = c.release();
    return CHEMK_OK;
}

extern "C" void chemk_ctx_free(chemk_ctx *c) {
    if (!c) return;
    hipSetDevice(c->device);
    for (auto &kv : c->graphs) hipGraphExecDestroy(kv.second);
    ann_destroy(c->ann);
    transport_destroy(c->transport);
    hipFree(c->tables);
    hipFree(c->bin);
    hipFree(c->queue);
    hipFree(c->small);
    hipFree(c->stats);
    delete c;
}

static int ensure_capacity(chemk_ctx *c, int64_t n) {
    if (n <= c->cap) return CHEMK_OK;
    hipFree(c->bin);
    hipFree(c->queue);
    c->bin = c->queue = nullptr;
    c->cap = 0;
    if (hipMalloc(&c->bin, sizeof(int) * n) != hipSuccess ||
        hipMalloc(&c->queue, sizeof(int) * n) != hipSuccess)
        return fail(CHEMK_E_OOM, "hipMalloc of DI queues for %lld cells failed", (long long)n);
    c->cap = n;
    // graphs captured with the old queues are stale
    for (auto &kv : c->graphs) hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    return CHEMK_OK;
}

// ---------------------------------------------------------------------------
// properties
// ---------------------------------------------------------------------------
static int check_n(int64_t n) {
    if (n < 0) return fail(CHEMK_E_ARG, "n=%lld < 0", (long long)n);
    if (n > (int64_t)std::numeric_limits<int>::max())
        return fail(CHEMK_E_UNSUPPORTED, "n=%lld above 2^31-1", (long long)n);
    return CHEMK_OK;
}

extern "C" int chemk_thermo(chemk_ctx *c, int64_t n, const double *T, const double *Y,
                            double *cp, double *h, void *stream) {
    g_err.clear();
    if (!c) return fail(CHEMK_E_ARG, "null context");
    if (int r = check_n(n)) return r;
    if (n == 0) return CHEMK_OK;
    if (!T || !Y || !cp || !h) return fail(CHEMK_E_ARG, "null array");
    if (int r = set_device(c)) return r;
    HIP_TRY(launch_thermo(c->dm, n, T, Y, cp, h, (hipStream_t)stream));
    return CHEMK_OK;
}

extern "C" int chemk_T_from_h(chemk_ctx *c, int64_t n, const double *h, const double *Y,
                              double *T, int32_t *status, void *stream) {
    g_err.clear();
    if (!c) return fail(CHEMK_E_ARG, "null context");
    if (int r = check_n(n)) return r;
    if (n == 0) return CHEMK_OK;
    if (!T || !Y || !h || !status) return fail(CHEMK_E_ARG, "null array");
    if (int r = set_device(c)) return r;
    HIP_TRY(launch_T_from_h(c->dm, n, h, Y, T, status, (hipStream_t)stream));
    return CHEMK_OK;
}

extern "C" int chemk_rhs(chemk_ctx *c, int64_t n, const double *T, const double *p,
                         const double *Y, double *dydt, void *stream) {
    g_err.clear();
    if (!c) return fail(CHEMK_E_ARG, "null context");
    if (int r = check_n(n)) return r;
    if (n == 0) return CHEMK_OK;
    if (!T || !p || !Y || !dydt) return fail(CHEMK_E_ARG, "null array");
    if (int r = set_device(c)) return r;
    HIP_TRY(launch_rhs(c->dm, n, T, p, Y, dydt, (hipStream_t)stream));
    return CHEMK_OK;
}

extern "C" int chemk_jacobian(chemk_ctx *c, int64_t n, const double *T, const double *p,
                              const double *Y, double *J, void *stream) {
    g_err.clear();
    if (!c) return fail(CHEMK_E_ARG, "null context");
    if (int r = check_n(n)) return r;
    if (n == 0) return CHEMK_OK;
    if (!T || !p || !Y || !J) return fail(CHEMK_E_ARG, "null array");
    if (int r = set_device(c)) return r;
    HIP_TRY(launch_jacobian(c->dm, n, T, p, Y, J, (hipStream_t)stream));
    return CHEMK_OK;
}

// ---------------------------------------------------------------------------
// advance
// ---------------------------------------------------------------------------
extern "C" void chemk_opts_default(chemk_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->mode = CHEMK_MODE_DI;
    o->max_steps = 100000;
    o->rtol = 1e-7;
    o->atol_Y = 1e-14;
    o->atol_T = 1e-6;
    o->h0_frac = 1e-3;
    o->bins = 0;
    o->waves_per_cu = 0;
    o->use_graph = 0;
    o->project = 1;
}

static int check_opts(const chemk_ctx *c, const chemk_opts *o) {
    if (!o) return fail(CHEMK_E_ARG, "null options");
    if (o->mode != CHEMK_MODE_DI && o->mode != CHEMK_MODE_ANN)
        return fail(CHEMK_E_ARG, "mode=%d unknown", o->mode);
    if (!(o->rtol > 0 && o->rtol < 1)) return fail(CHEMK_E_ARG, "rtol must be in (0, 1)");
    if (!(o->atol_Y >= 0) || !(o->atol_T >= 0)) return fail(CHEMK_E_ARG, "atol must be >= 0");
    if (!(o->h0_frac > 0 && o->h0_frac <= 1)) return fail(CHEMK_E_ARG, "h0_frac must be in (0, 1]");
    if (o->max_steps < 1) return fail(CHEMK_E_ARG, "max_steps must be >= 1");
    if (o->bins < 0 || o->bins > kMaxBins)
        return fail(CHEMK_E_ARG, "bins=%d outside [0, %d]", o->bins, kMaxBins);
    if (o->waves_per_cu < 0 || o->waves_per_cu > 32)
        return fail(CHEMK_E_ARG, "waves_per_cu=%d outside [0, 32]", o->waves_per_cu);
    if (o->di_kernel != CHEMK_DI_AUTO && o->di_kernel != CHEMK_DI_LDS_LU && o->di_kernel != CHEMK_DI_REG_LU)
        return fail(CHEMK_E_ARG, "di_kernel=%d unknown", o->di_kernel);
    if (o->di_kernel == CHEMK_DI_REG_LU && !di_has_reg_lu(c->dm.N))
        return fail(CHEMK_E_ARG, "no register-LU DI kernel for N = %d (it exists for 10 and 33)", c->dm.N);
    return CHEMK_OK;
}

// The DI factorisation: the caller's, else the tuned one, else automatic.
static int resolve_variant(const chemk_ctx *c, const chemk_opts *o) {
    return o->di_kernel != CHEMK_DI_AUTO ? o->di_kernel : c->tuned_variant;
}

static void resolve_tuning(const chemk_ctx *c, const chemk_opts *o, int &bins, int &wpc) {
    bins = o->bins > 0 ? o->bins : (c->tuned_bins > 0 ? c->tuned_bins : 16);
    wpc = o->waves_per_cu > 0 ? o->waves_per_cu : (c->tuned_wpc > 0 ? c->tuned_wpc : 8);
}

// Device scratch of one DI step: stiffness bins and queue [n], the small
// counters (queue counter, item count, histogram, offsets) and statistics.
struct DiScratch {
    int *bin, *queue, *small;
    unsigned long long *stats;
};

static DiScratch ctx_scratch(chemk_ctx *c) { return DiScratch{c->bin, c->queue, c->small, c->stats}; }

// Enqueue the DI step over all n cells.  queue order from the stiffness bins.
static int enqueue_di(chemk_ctx *c, const DiScratch &w, int64_t n, double *T, const double *p, double *Y,
                      double dt, const chemk_opts *o, int bins, int wpc, int32_t *status, int32_t *nsteps,
                      hipStream_t s, bool timed = true) {
    int *counter = w.small, *n_items = w.small + 1;
    int *hist = w.small + 2, *offs = w.small + 2 + kMaxBins;
    HIP_TRY(launch_zero_u64(w.stats, 4, s));
    HIP_TRY(launch_zero_ints(counter, 1, s));
    HIP_TRY(launch_set_int(n_items, (int)n, s));
    const int *queue = nullptr;
    if (bins > 1) {
        if (timed) c->timer.begin(CHEMK_PHASE_BINNING, s);
        HIP_TRY(launch_binning(c->dm, (int)n, T, p, Y, dt, bins, w.bin, hist, offs, w.queue, s));
        if (timed) c->timer.end(CHEMK_PHASE_BINNING, s);
        queue = w.queue;
    }
    const int64_t grid64 = std::min<int64_t>(n, (int64_t)c->cu_count * wpc);
    if (timed) c->timer.begin(CHEMK_PHASE_DI, s);
    HIP_TRY(launch_di(c->dm, (int)grid64, n_items, queue, counter, T, p, Y, dt, o->rtol,
                      o->atol_Y, o->atol_T, o->h0_frac, o->max_steps, o->project, status, nsteps,
                      w.stats, 0, resolve_variant(c, o), s));
    if (timed) c->timer.end(CHEMK_PHASE_DI, s);
    c->last_stats = w.stats;
    return CHEMK_OK;
}

extern "C" int chemk_advance(chemk_ctx *c, int64_t n, double *T, const double *p, double *Y,
                             double dt, const chemk_opts *o, int32_t *status, int32_t *nsteps,
                             void *stream) {
    g_err.clear();
    if (!c) return fail(CHEMK_E_ARG, "null context");
    if (int r = check_n(n)) return r;
    if (int r = check_opts(c, o)) return r;
    if (!(dt > 0) || !std::isfinite(dt)) return fail(CHEMK_E_ARG, "dt must be finite and > 0");
    if (n == 0) return CHEMK_OK;
    if (!T || !p || !Y || !status) return fail(CHEMK_E_ARG, "null array");
    if (o->mode == CHEMK_MODE_ANN) {
        if (!c->ann || !ann_ready(c->ann))
            return fail(CHEMK_E_STATE, "ANN mode needs chemk_ann_create, weights and norm first");
        const double tdt = ann_dt(c->ann);
        if (!(std::fabs(dt - tdt) <= 1e-12 * std::fabs(tdt)))
            return fail(CHEMK_E_DT, "dt=%.17g differs from the trained dt=%.17g", dt, tdt);
    }
    if (int r = set_device(c)) return r;
    if (int r = ensure_capacity(c, n)) return r;
    hipStream_t s = (hipStream_t)stream;
    int bins, wpc;
    resolve_tuning(c, o, bins, wpc);
    c->last_stats = c->stats;

    auto enqueue = [&]() -> int {
        if (o->mode == CHEMK_MODE_DI)
            return enqueue_di(c, ctx_scratch(c), n, T, p, Y, dt, o, bins, wpc, status, nsteps, s);
        AnnStepArgs a{n, T, p, Y, dt, o->rtol, o->atol_Y, o->atol_T, o->h0_frac, o->max_steps,
                      o->project, resolve_variant(c, o), status, nsteps, c->cu_count * wpc, c->queue, c->small,
                      c->small + 1, c->stats, &c->dm, &c->timer, bins, c->bin, c->small + 2,
                      c->small + 2 + kMaxBins};
        hipError_t e = ann_enqueue_step(c->ann, a, s);
        if (e != hipSuccess)
            return fail(CHEMK_E_HIP, "ANN step: %s", hipGetErrorString(e));
        c->last_stats = c->stats;
        return CHEMK_OK;
    };
    if (o->mode == CHEMK_MODE_ANN) {
        // buffers and tables first: nothing is allocated inside a capture
        hipError_t e = ann_prepare(c->ann, c->dm, n, s);
        if (e != hipSuccess) return fail(CHEMK_E_HIP, "ANN step set-up: %s", hipGetErrorString(e));
    }
    if (!o->use_graph || c->timer.on) return enqueue();

    const uint64_t gen = o->mode == CHEMK_MODE_ANN ? ann_generation(c->ann) : 0;
    GraphKey key{n, T, p, Y, status, nsteps, dt, o->mode, bins, wpc, o->max_steps, o->project,
                 o->rtol, o->atol_Y, o->atol_T, o->h0_frac, gen};
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        // graphs of an earlier network state can never be replayed again
        for (auto g = c->graphs.begin(); g != c->graphs.end();) {
            if (g->first.mode == CHEMK_MODE_ANN && g->first.ann_gen != gen) {
                hipGraphExecDestroy(g->second);
                g = c->graphs.erase(g);
            } else {
                ++g;
            }
        }
        hipStream_t cs = s;
        hipStream_t own = nullptr;
        if (!cs) {   // capture needs a non-default stream
            HIP_TRY(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
            cs = own;
        }
        HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        hipStream_t saved = s;
        s = cs;
        int r = enqueue();
        s = saved;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(cs, &g);
        if (own) hipStreamDestroy(own);
        if (r) {
            if (g) hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess) return fail(CHEMK_E_HIP, "graph capture: %s", hipGetErrorString(e));
        hipGraphExec_t ge = nullptr;
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) return fail(CHEMK_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
        it = c->graphs.emplace(key, ge).first;
    }
    HIP_TRY(hipGraphLaunch(it->second, s));
    return CHEMK_OK;
}

extern "C" int chemk_advance_noalloc(chemk_ctx *c, int64_t n, double *T, const double *p, double *Y,
                                     double dt, const chemk_opts *o, int32_t *status, int32_t *nsteps,
                                     void *stream) {
    g_err.clear();
    if (!c) return fail(CHEMK_E_ARG, "null context");
    if (int r = check_n(n)) return r;
    if (n > CHEMK_NOALLOC_MAX_CELLS)
        return fail(CHEMK_E_ARG, "n=%lld above CHEMK_NOALLOC_MAX_CELLS=%d of the no-allocation advance",
                    (long long)n, CHEMK_NOALLOC_MAX_CELLS);
    if (int r = check_opts(c, o)) return r;
    if (o->mode != CHEMK_MODE_DI) return fail(CHEMK_E_ARG, "the no-allocation advance is DI mode only");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(CHEMK_E_ARG, "dt must be finite and > 0");
    if (n == 0) return CHEMK_OK;
    if (!T || !p || !Y || !status) return fail(CHEMK_E_ARG, "null array");
    if (!c->noalloc) return fail(CHEMK_E_STATE, "no-allocation scratch not set up");
    if (int r = set_device(c)) return r;
    int bins, wpc;
    resolve_tuning(c, o, bins, wpc);
    unsigned char *base = static_cast<unsigned char *>(c->noalloc);
    DiScratch w{reinterpret_cast<int *>(base + kNaBin), reinterpret_cast<int *>(base + kNaQueue),
                reinterpret_cast<int *>(base + kNaSmall), reinterpret_cast<unsigned long long *>(base)};
    return enqueue_di(c, w, n, T, p, Y, dt, o, bins, wpc, status, nsteps, (hipStream_t)stream, false);
}

extern "C" int chemk_last_counters(chemk_ctx *c, int64_t out[3], void *stream) {
    g_err.clear();
    if (!c || !out) return fail(CHEMK_E_ARG, "null argument");
    if (int r = set_device(c)) return r;
    unsigned long long h[4];
    HIP_TRY(hipMemcpyAsync(h, c->last_stats ? c->last_stats : c->stats, sizeof h, hipMemcpyDeviceToHost,
                           (hipStream_t)stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    for (int i = 0; i < 3; ++i) out[i] = (int64_t)h[i];
    return CHEMK_OK;
}

extern "C" int chemk_timing(chemk_ctx *c, int32_t enable) {
    g_err.clear();
    if (!c) return fail(CHEMK_E_ARG, "null context");
    c->timer.on = enable != 0;
    return CHEMK_OK;
}

extern "C" int chemk_timing_read(chemk_ctx *c, double ms[CHEMK_NUM_PHASES],
                                 int64_t launches[CHEMK_NUM_PHASES], void *stream) {
    g_err.clear();
    if (!c || !ms || !launches) return fail(CHEMK_E_ARG, "null argument");
    if (int r = set_device(c)) return r;
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    for (int p = 0; p < CHEMK_NUM_PHASES; ++p) {
        double acc = 0.0;
        for (auto &pr : c->timer.done[p]) {
            float t = 0.f;
            HIP_TRY(hipEventElapsedTime(&t, pr.first, pr.second));
            acc += t;
        }
        ms[p] = acc;
        launches[p] = (int64_t)c->timer.done[p].size();
    }
    c->timer.release_all();
    return CHEMK_OK;
}

// ---------------------------------------------------------------------------
// autotuner: grid over (bins, waves per CU), then the DI factorisation, on
// copies of the state; results cached per (arch, CUs, K, R, E, log2 n)
// ---------------------------------------------------------------------------
namespace {
struct TuneKey {
    std::string arch;
    int cu, K, R, E, nlog2;
    bool operator<(const TuneKey &o) const {
        return std::tie(arch, cu, K, R, E, nlog2) < std::tie(o.arch, o.cu, o.K, o.R, o.E, o.nlog2);
    }
};
struct TuneVal {
    int bins, wpc, variant;
    double ms;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
std::string g_tune_loaded;   // the CHEMK_TUNE_CACHE file read into g_tune

// Cache file: one entry per line, "arch cu K R E nlog2 bins wpc variant ms".
void tune_file_load(const std::string &path) {
    std::ifstream f(path);
    TuneKey k;
    TuneVal v;
    while (f >> k.arch >> k.cu >> k.K >> k.R >> k.E >> k.nlog2 >> v.bins >> v.wpc >> v.variant >> v.ms)
        if (v.bins >= 1 && v.bins <= 256 && v.wpc >= 1 && v.wpc <= 32 && v.variant >= 0 && v.variant <= 2)
            g_tune.emplace(k, v);
}

void tune_file_save(const std::string &path) {
    std::ofstream f(path, std::ios::trunc);
    for (const auto &kv : g_tune)
        f << kv.first.arch << ' ' << kv.first.cu << ' ' << kv.first.K << ' ' << kv.first.R << ' ' << kv.first.E
          << ' ' << kv.first.nlog2 << ' ' << kv.second.bins << ' ' << kv.second.wpc << ' ' << kv.second.variant
          << ' ' << kv.second.ms << '\n';
}

std::string tune_file() {
    const char *e = std::getenv("CHEMK_TUNE_CACHE");
    return e ? std::string(e) : std::string();
}
}  // namespace

extern "C" void chemk_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    g_tune_loaded.clear();
}

extern "C" int chemk_tuning(chemk_ctx *c, int32_t out[3]) {
    g_err.clear();
    if (!c || !out) return fail(CHEMK_E_ARG, "null argument");
    out[0] = c->tuned_bins;
    out[1] = c->tuned_wpc;
    out[2] = c->tuned_variant;
    return CHEMK_OK;
}

extern "C" int chemk_autotune(chemk_ctx *c, int64_t n, const double *T, const double *p,
                              const double *Y, double dt, const chemk_opts *o, int32_t best[2],
                              double *best_ms, void *stream) {
    g_err.clear();
    if (!c || !best) return fail(CHEMK_E_ARG, "null argument");
    if (int r = check_n(n)) return r;
    if (int r = check_opts(c, o)) return r;
    if (n == 0 || !T || !p || !Y) return fail(CHEMK_E_ARG, "autotune needs cells");
    int nlog2 = 0;
    while ((int64_t(1) << (nlog2 + 1)) <= n) ++nlog2;
    const TuneKey key{c->arch, c->cu_count, c->K, c->R, c->E, nlog2};
    const std::string path = tune_file();
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (!path.empty() && g_tune_loaded != path) {
            tune_file_load(path);
            g_tune_loaded = path;
        }
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            c->tuned_bins = it->second.bins;
            c->tuned_wpc = it->second.wpc;
            c->tuned_variant = it->second.variant;
            best[0] = it->second.bins;
            best[1] = it->second.wpc;
            if (best_ms) *best_ms = it->second.ms;
            return CHEMK_OK;
        }
    }
    if (int r = set_device(c)) return r;
    if (int r = ensure_capacity(c, n)) return r;
    hipStream_t s = (hipStream_t)stream;
    const int K = c->K;
    double *Tc = nullptr, *Yc = nullptr;
    int *st = nullptr;
    if (hipMalloc(&Tc, 8 * n) != hipSuccess || hipMalloc(&Yc, 8 * n * K) != hipSuccess ||
        hipMalloc(&st, 4 * n) != hipSuccess) {
        hipFree(Tc);
        hipFree(Yc);
        hipFree(st);
        return fail(CHEMK_E_OOM, "autotune copies");
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int bins_grid[] = {1, 8, 32};
    const int wpc_grid[] = {4, 8, 12};
    double bestt = 1e300;
    int bb = 16, bw = 8, bv = CHEMK_DI_AUTO;
    chemk_opts oo = *o;
    oo.mode = CHEMK_MODE_DI;
    oo.use_graph = 0;
    int rc = CHEMK_OK;
    // one timed DI advance of the copies; returns its milliseconds or < 0
    auto trial = [&](int b, int w, int v) -> double {
        if (hipMemcpyAsync(Tc, T, 8 * n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(Yc, Y, 8 * n * K, hipMemcpyDeviceToDevice, s) != hipSuccess) {
            rc = fail(CHEMK_E_HIP, "autotune copy");
            return -1.0;
        }
        oo.di_kernel = v;
        hipEventRecord(e0, s);
        if ((rc = enqueue_di(c, ctx_scratch(c), n, Tc, p, Yc, dt, &oo, b, w, st, nullptr, s))) return -1.0;
        hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = fail(CHEMK_E_HIP, "autotune sync");
            return -1.0;
        }
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        return ms;
    };
    const int v0 = o->di_kernel;   // the caller's factorisation (automatic unless fixed)
    for (int b : bins_grid)
        for (int w : wpc_grid) {
            const double ms = trial(b, w, v0);
            if (ms < 0) goto done;
            if (ms < bestt) {
                bestt = ms;
                bb = b;
                bw = w;
                bv = v0;
            }
        }
    if (v0 == CHEMK_DI_AUTO && di_has_reg_lu(c->N)) {
        const double ms = trial(bb, bw, CHEMK_DI_LDS_LU);
        if (ms < 0) goto done;
        if (ms < bestt) {
            bestt = ms;
            bv = CHEMK_DI_LDS_LU;
        }
    }
    c->tuned_bins = bb;
    c->tuned_wpc = bw;
    c->tuned_variant = bv;
    best[0] = bb;
    best[1] = bw;
    if (best_ms) *best_ms = bestt;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = TuneVal{bb, bw, bv, bestt};
        if (!path.empty()) tune_file_save(path);
    }
done:
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(Tc);
    hipFree(Yc);
    hipFree(st);
    return rc;
}
