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
//   sincos_half_turn(t)  sin(pi t), cos(pi t) for t in [0, 2]: k = rint(t),
//                   r = t - k in [-1/2, 1/2] exactly, Taylor series of
//                   sin(pi r) to r^21 and cos(pi r) to r^20 (truncation below
//                   2e-17), coefficients rounded from 70-digit values of
//                   pi^n / n!; an odd k negates both results.
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

// sqrt x for x >= 0 (0 gives 0: the seed is taken at a tiny positive
// number and every correction then stays exactly 0).
__host__ __device__ __forceinline__ double sqrt_pos(double x) {
#pragma clang fp contract(off)
    const double y = rsq_seed(__builtin_fmax(x, 0x1p-1000));
    double g = x * y;      // ~ sqrt x
    double h = 0.5 * y;    // ~ 1 / (2 sqrt x)
    const double e = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, e, g);
    h = __builtin_fma(h, e, h);
    double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    return g;
}

// sin(pi t) -> s, cos(pi t) -> c, for t in [0, 2].
__host__ __device__ __forceinline__ void sincos_half_turn(double t, double &s, double &c) {
#pragma clang fp contract(off)
    const double k = __builtin_rint(t);  // 0, 1 or 2
    const double r = t - k;             // exact, in [-1/2, 1/2]
    const double r2 = r * r;
    double ps = 5.392664662608129e-10;
    ps = __builtin_fma(ps, r2, -2.2948428997269873e-08);
    ps = __builtin_fma(ps, r2, 7.952054001475513e-07);
    ps = __builtin_fma(ps, r2, -2.1915353447830217e-05);
    ps = __builtin_fma(ps, r2, 0.00046630280576761255);
    ps = __builtin_fma(ps, r2, -0.0073704309457143504);
    ps = __builtin_fma(ps, r2, 0.08214588661112823);
    ps = __builtin_fma(ps, r2, -0.5992645293207921);
    ps = __builtin_fma(ps, r2, 2.5501640398773455);
    ps = __builtin_fma(ps, r2, -5.16771278004997);
    ps = __builtin_fma(ps, r2, 3.141592653589793);
    double pc = 3.604730797462501e-09;
    pc = __builtin_fma(pc, r2, -1.3878952462213771e-07);
    pc = __builtin_fma(pc, r2, 4.303069587032947e-06);
    pc = __builtin_fma(pc, r2, -0.0001046381049248457);
    pc = __builtin_fma(pc, r2, 0.0019295743094039231);
    pc = __builtin_fma(pc, r2, -0.02580689139001406);
    pc = __builtin_fma(pc, r2, 0.2353306303588932);
    pc = __builtin_fma(pc, r2, -1.3352627688545895);
    pc = __builtin_fma(pc, r2, 4.0587121264167685);
    pc = __builtin_fma(pc, r2, -4.934802200544679);
    pc = __builtin_fma(pc, r2, 1.0);
    // an odd number of half turns negates both
    const uint64_t flip = (uint64_t)((int)k & 1) << 63;
    s = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, r * ps) ^ flip);
    c = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, pc) ^ flip);
}

}  // namespace pr
