// Known-good and known-bad shapes for the wave-convergence check.  Compiled
// to device IR only; never launched.
#include <hip/hip_runtime.h>

// A queue claim by lane 0 inside a lane-0 branch, broadcast with
// readfirstlane, and a lane-0 epilogue at the end of the iteration.
__global__ void __launch_bounds__(64) claim_lane0_branch(int *counter, int n, int *out) {
    const int lane = threadIdx.x & 63;
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(counter, 1);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= n) break;
        out[item * 64 + lane] += lane;
        if (lane == 0) out[item * 64] = -1;
    }
}

// The same queue with the claim issued by every lane.
__global__ void __launch_bounds__(64) claim_all_lanes(int *counter, int n, int *out) {
    const int lane = threadIdx.x & 63;
    for (;;) {
        const int got = atomicAdd(counter, lane == 0 ? 1 : 0);
        const int item = __builtin_amdgcn_readfirstlane(got);
        if (item >= n) break;
        out[item * 64 + lane] += lane;
        if (lane == 0) out[item * 64] = -1;
    }
}

__device__ __forceinline__ double butterfly(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Newton-like loop whose exit test uses a butterfly sum as is.
__global__ void __launch_bounds__(64) exit_on_butterfly(const double *a, double *out) {
    const int lane = threadIdx.x & 63;
    double x = 1.0;
    for (int it = 0; it < 50; ++it) {
        const double f = butterfly(a[lane] * x) - 1.0;
        x -= f;
        if (fabs(f) < 1e-12) break;
    }
    out[lane] = x;
}

// The same loop with the sum broadcast from the first lane.
__global__ void __launch_bounds__(64) exit_on_broadcast(const double *a, double *out) {
    const int lane = threadIdx.x & 63;
    double x = 1.0;
    for (int it = 0; it < 50; ++it) {
        const double s = butterfly(a[lane] * x);
        const int lo = __builtin_amdgcn_readfirstlane(__double2loint(s));
        const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(s));
        const double f = __hiloint2double(hi, lo) - 1.0;
        x -= f;
        if (fabs(f) < 1e-12) break;
    }
    out[lane] = x;
}

// A loop over groups of lanes that leaves when no lane's predicate holds: the
// ballot of the predicate is the same mask on every lane.
__global__ void __launch_bounds__(64) exit_on_ballot(const double *a, double *out) {
    const int lane = threadIdx.x & 63;
    double x = a[lane];
    for (int it = 0; it < 8; ++it) {
        x = 0.5 * (x + butterfly(x) / 64.0);
        const bool more = x > 1.0;
        if (!__ballot(more)) break;
    }
    out[lane] = x;
}
