// dpk_device.h -- device helpers shared by the embedding kernels (network and table paths).
#pragma once
#include <hip/hip_runtime.h>

namespace dpk {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Wave-scope ordering of LDS traffic between lanes of one wave.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Switching function of Sec. II.A.1 (eq. switch) and its derivative, FP64, from r, ir = 1/r and
// inv_w = 1/(rc - rs) (no division here: the caller's 1/r is the only one per neighbour).
__device__ __forceinline__ void switch_fn(double r, double ir, double rs, double rc, double inv_w, double& s,
                                          double& ds)
{
    if (r < rs) {
        s = ir;
        ds = -ir * ir;
    } else if (r < rc) {
        // u = x^3 (-6 x^2 + 15 x - 10) + 1 as (1 - x)^3 (1 + 3 x + 6 x^2): no cancellation near
        // r_c, so s >= 0 (a table counts negative inputs as out of range)
        double x = (r - rs) * inv_w;
        double y = 1.0 - x;
        double u = y * y * y * (1.0 + x * (3.0 + 6.0 * x));
        double du = -30.0 * x * x * y * y;
        s = u * ir;
        ds = du * ir * inv_w - u * ir * ir;
    } else {
        s = 0.0;
        ds = 0.0;
    }
}

}  // namespace dpk
