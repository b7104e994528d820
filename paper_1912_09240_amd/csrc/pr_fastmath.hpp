// FP64 helpers of the Box-Muller transform of the fine propagator:
//
//   sqrt_pos(x)          square root, x >= 0: hardware reciprocal-sqrt seed and
//                        two Newton-Raphson corrections; within 1 ulp.
//   sqrt_positive(x)     the same steps for x > 0 (normal numbers), without
//                        the clamp that makes sqrt_pos(0) = 0.
//   mantissa_exponent(u) u = m 2^e with m in [1/2, 1) (frexp).
//
// Each has a host form (C library seeds) so that the tests can run the same
// arithmetic on the CPU.
#pragma once

#include <hip/hip_runtime.h>

namespace pr {

__host__ __device__ __forceinline__ double rsq_seed(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsq(x);
#else
    return 1.0 / __builtin_sqrt(x);
#endif
}

__host__ __device__ __forceinline__ double mantissa_exponent(double u, int &e) {
#if defined(__HIP_DEVICE_COMPILE__)
    e = __builtin_amdgcn_frexp_exp(u);
    return __builtin_amdgcn_frexp_mant(u);
#else
    return __builtin_frexp(u, &e);
#endif
}

// Two Newton-Raphson corrections g += (x - g^2) h of g = x y, h = y/2, from
// a reciprocal-sqrt seed y of x.  The hardware seed is good to ~2^-24
// relative, so the first correction leaves ~1.5 (2^-24)^2 and the second
// ~2^-47 x 2^-24: the result is within the rounding of its last fma.
__host__ __device__ __forceinline__ double sqrt_from_seed(double x, double y) {
#pragma clang fp contract(off)
    double g = x * y;      // ~ sqrt x
    const double h = 0.5 * y;  // ~ 1 / (2 sqrt x)
    double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    return g;
}

// sqrt x for x >= 0 (0 gives 0: the seed is taken at a tiny positive
// number and every correction then stays exactly 0).
__host__ __device__ __forceinline__ double sqrt_pos(double x) {
    return sqrt_from_seed(x, rsq_seed(__builtin_fmax(x, 0x1p-1000)));
}

// sqrt x for normal x > 0.
__host__ __device__ __forceinline__ double sqrt_positive(double x) { return sqrt_from_seed(x, rsq_seed(x)); }

}  // namespace pr
