// chemk_internal.h -- host-side declarations shared by the library's sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chemk.h"

#include <utility>
#include <vector>

#define CHEMK_MAX_ELEMENTS_DEV CHEMK_MAX_ELEMENTS

namespace chemk {

// HIP-event brackets around the launches of each phase (profiling aid).
struct PhaseTimer {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> done[CHEMK_NUM_PHASES];
    hipEvent_t open[CHEMK_NUM_PHASES] = {};
    std::vector<hipEvent_t> pool;

    hipEvent_t take() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        // Timing only (read after a stream synchronize): no system-scope
        // fence, whose cache writeback would slow the launches that follow.
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
        return e;
    }
    void begin(int ph, hipStream_t s) {
        if (!on) return;
        open[ph] = take();
        if (open[ph]) (void)hipEventRecord(open[ph], s);
    }
    void end(int ph, hipStream_t s) {
        if (!on || !open[ph]) return;
        hipEvent_t e = take();
        if (!e) return;
        (void)hipEventRecord(e, s);
        done[ph].push_back({open[ph], e});
        open[ph] = nullptr;
    }
    void release_all() {
        for (int p = 0; p < CHEMK_NUM_PHASES; ++p) {
            for (auto &pr : done[p]) {
                pool.push_back(pr.first);
                pool.push_back(pr.second);
            }
            done[p].clear();
        }
    }
    ~PhaseTimer() {
        release_all();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

struct DevMech;

// di.hip
int di_template_N(int Nreal);
size_t di_lds_bytes(int K, int R, int N);
size_t di_block_lds_bytes(int K, int R);   // LDS of one DI workgroup
hipError_t launch_di(const DevMech &m, int grid, const int *n_items, const int *queue,
                     int *counter, double *T, const double *p, double *Y, double dt,
                     double rtol, double atolY, double atolT, double h0_frac, int max_steps,
                     int project, int *status, int *nsteps, unsigned long long *stats,
                     int status_or, int variant, hipStream_t s);
bool di_has_reg_lu(int N);
void transport_destroy(void *t);
hipError_t launch_binning(const DevMech &m, int n, const double *T, const double *p,
                          const double *Y, double dt, int bins, int *bin, int *hist, int *offs,
                          int *queue, hipStream_t s);
// Binning of the cells idx[0 .. *count) (count on the device, at most n_max):
// queue receives them ordered by the stiffness key, most active bin first.
hipError_t launch_binning_list(const DevMech &m, int n_max, const int *count, const int *idx,
                               const double *T, const double *p, const double *Y, double dt, int bins,
                               int *bin, int *hist, int *offs, int *queue, hipStream_t s);
hipError_t launch_zero_ints(int *p, int n, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s);
hipError_t launch_set_int(int *p, int v, hipStream_t s);

// props.hip
hipError_t launch_thermo(const DevMech &m, int64_t n, const double *T, const double *Y,
                         double *cp, double *h, hipStream_t s);
hipError_t launch_T_from_h(const DevMech &m, int64_t n, const double *h, const double *Y,
                           double *T, int *status, hipStream_t s);
hipError_t launch_rhs(const DevMech &m, int64_t n, const double *T, const double *p,
                      const double *Y, double *dydt, hipStream_t s);
hipError_t launch_jacobian(const DevMech &m, int64_t n, const double *T, const double *p,
                           const double *Y, double *J, hipStream_t s);

}  // namespace chemk
