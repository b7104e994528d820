// FP64 elementary functions for the Box-Muller transform of the fine
// propagator, written for the VALU budget of one Euler-Maruyama step: the
// arguments are known to lie in small ranges, so no general-purpose reduction
// is needed.
//
//   log_unit(u)     natural logarithm for u in (0, 1]:
//                   u = m 2^e with m in [1/sqrt 2, sqrt 2), s = (m-1)/(m+1),
//                   ln m = 2 atanh s = 2s + s z (2/3 + 2z/5 + ... + 2z^8/19),
//                   z = s^2 <= 0.0295 (truncation below 4e-16 relative);
//                   ln u = e ln2 + ln m with ln 2 split in an exact high part.
//   sqrt_pos(x)     square root, x >= 0: hardware reciprocal-sqrt seed and
//                   Newton-Raphson (Goldschmidt form) steps.
//   sincos_quarter(t)  sin(pi t / 2), cos(pi t / 2) for t in [0, 4]: quadrant
//                   k = rint(t), r = t - k in [-1/2, 1/2] exactly, then the
//                   Taylor series of sin(pi r/2) to r^15 and cos(pi r/2) to
//                   r^16 (truncation below 7e-17), coefficients rounded from
//                   70-digit values of (pi/2)^n / n!.
//
// All three are within a few ulp of the correctly rounded results; the
// Box-Muller normals they produce match those of a C library to ~1e-15.
#pragma once

#include <hip/hip_runtime.h>

namespace pr {

__host__ __device__ __forceinline__ double rcp_seed(double d) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcp(d);
#else
    return 1.0 / d;
#endif
}

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

// ln u for u in (0, 1].
__host__ __device__ __forceinline__ double log_unit(double u) {
#pragma clang fp contract(off)
    int e;
    double m = mantissa_exponent(u, e);  // m in [1/2, 1)
    if (m < 0.7071067811865476) {
        m = m + m;
        e -= 1;
    }
    const double f = m - 1.0;  // exact
    const double d = 2.0 + f;
    double r = rcp_seed(d);
    r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
    r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
    double s = f * r;
    s = __builtin_fma(r, __builtin_fma(-d, s, f), s);  // s = f / (2 + f)
    const double z = s * s;
    double p = 0.10526315789473684;  // 2/19
    p = __builtin_fma(p, z, 0.11764705882352941);  // 2/17
    p = __builtin_fma(p, z, 0.13333333333333333);  // 2/15
    p = __builtin_fma(p, z, 0.15384615384615385);  // 2/13
    p = __builtin_fma(p, z, 0.18181818181818182);  // 2/11
    p = __builtin_fma(p, z, 0.2222222222222222);   // 2/9
    p = __builtin_fma(p, z, 0.2857142857142857);   // 2/7
    p = __builtin_fma(p, z, 0.4);                  // 2/5
    p = __builtin_fma(p, z, 0.6666666666666666);   // 2/3
    const double lnm = __builtin_fma(s * z, p, s + s);
    const double ed = (double)e;
    return __builtin_fma(ed, 0.6931471803691238, __builtin_fma(ed, 1.9082149292705877e-10, lnm));
}

// sqrt x for x >= 0 (0 gives 0).
__host__ __device__ __forceinline__ double sqrt_pos(double x) {
#pragma clang fp contract(off)
    const double y = rsq_seed(x > 0.0 ? x : 1.0);
    double g = x * y;      // ~ sqrt x
    double h = 0.5 * y;    // ~ 1 / (2 sqrt x)
    const double e = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, e, g);
    h = __builtin_fma(h, e, h);
    double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    return x > 0.0 ? g : 0.0;
}

// sin(pi t/2) -> s, cos(pi t/2) -> c, for t in [0, 4].
__host__ __device__ __forceinline__ void sincos_quarter(double t, double &s, double &c) {
#pragma clang fp contract(off)
    const double k = __builtin_rint(t);
    const double r = t - k;  // exact
    const double r2 = r * r;
    double ps = -6.688035109811468e-10;
    ps = __builtin_fma(ps, r2, 5.692172921967927e-08);
    ps = __builtin_fma(ps, r2, -3.598843235212085e-06);
    ps = __builtin_fma(ps, r2, 0.00016044118478735983);
    ps = __builtin_fma(ps, r2, -0.004681754135318688);
    ps = __builtin_fma(ps, r2, 0.07969262624616705);
    ps = __builtin_fma(ps, r2, -0.6459640975062463);
    ps = __builtin_fma(ps, r2, 1.5707963267948966);
    const double sn = r * ps;
    double pc = 6.565963114979473e-11;
    pc = __builtin_fma(pc, r2, -6.386603083791852e-09);
    pc = __builtin_fma(pc, r2, 4.710874778818172e-07);
    pc = __builtin_fma(pc, r2, -2.5202042373060607e-05);
    pc = __builtin_fma(pc, r2, 0.0009192602748394266);
    pc = __builtin_fma(pc, r2, -0.02086348076335296);
    pc = __builtin_fma(pc, r2, 0.25366950790104803);
    pc = __builtin_fma(pc, r2, -1.2337005501361697);
    const double cs = __builtin_fma(pc, r2, 1.0);
    const int q = (int)k & 3;
    const double a = (q & 1) ? cs : sn;  // |sin| part
    const double b = (q & 1) ? sn : cs;  // |cos| part
    s = (q & 2) ? -a : a;
    c = ((q + 1) & 2) ? -b : b;
}

}  // namespace pr
