// ann_internal.h -- the learned part's state and step enqueue (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chemk {
struct DevMech;
struct PhaseTimer;
}

struct AnnState;

struct AnnStepArgs {
    int64_t n;
    double *T;
    const double *p;
    double *Y;
    double dt, rtol, atolY, atolT, h0_frac;
    int max_steps, project, di_kernel;
    int32_t *status, *nsteps;
    int di_grid;
    int *queue;              // [n] routed cells
    int *counter, *n_routed; // device ints
    unsigned long long *stats;
    const chemk::DevMech *dm;
    chemk::PhaseTimer *timer;
    int bins;                    // stiffness bins of the routed cells (<= 1: queue order)
    int *bin, *hist, *offs;      // binning scratch: [n], [bins], [bins]
};

void ann_destroy(AnnState *a);
bool ann_ready(const AnnState *a);
double ann_dt(const AnnState *a);
hipError_t ann_enqueue_step(AnnState *a, const AnnStepArgs &args, hipStream_t s);
hipError_t ann_prepare(AnnState *a, const chemk::DevMech &m, int64_t n, hipStream_t s);
uint64_t ann_generation(const AnnState *a);
