// How an adjoint reads dL/dy beyond a plain trajectory-shaped g (the
// neural-ODE and block solvers): every entry divided by a device scalar (the
// Frobenius loss's g = y / L read straight from the trajectory, so g is never
// formed), and/or g given at the observed steps only (Appendix A: dL/dy
// enters the adjoint only where the loss observes the state).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace tvi {

struct GradInput {
    const double *div;   // device scalar dividing every entry of g, or null
    const int32_t *obs;  // observed steps, strictly increasing (uniform grids), or null
    int32_t n_obs;       // their number (>= 1 with obs)
};

__device__ __forceinline__ double grad_scale(const GradInput &gi) { return gi.div ? 1.0 / *gi.div : 1.0; }

// dL/dy at step k of series b (first point p0): g's entry in the trajectory
// layout, or with observed steps (g [B][n_obs][n]) the row of the observation
// at step k, found by bisection; null where step k is not observed (dL/dy_k = 0).
template <class IO>
__device__ __forceinline__ const IO *grad_at(const IO *g, const GradInput &gi, int64_t b, int64_t p0, int64_t k, int n)
{
    if (!gi.obs) return g + (p0 + k) * n;
    int lo = 0, hi = gi.n_obs;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (gi.obs[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return (lo < gi.n_obs && gi.obs[lo] == k) ? g + (b * gi.n_obs + lo) * n : nullptr;
}

} // namespace tvi
