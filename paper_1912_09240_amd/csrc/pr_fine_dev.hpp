// Device side of the fine propagator shared by the single-instance and the
// batched launches: the scheme's coefficients and one Euler-Maruyama step
// (Sec. 2.1.3 eq. (EMx)/(EMy)) of one particle with its in-kernel normals.
#pragma once

#include <cmath>

#include "pr_internal.hpp"

namespace pr {

// Parameters of the scheme, precomputed on the host.
template <typename T>
struct EmCoef {
    T a3, a1, al;  // -dt times the drift coefficients of X: c3 x^3 + c1 x + lam (x - ybar)
    T rate;        // dt / eps
    T sx;          // sqrt(2 dt / beta)
    T sy;          // sqrt(2 dt / (beta eps))
};

template <typename T>
__device__ __forceinline__ void normal_pair(const NoiseTab &tab, Key key, uint32_t inst, uint32_t tag,
                                            uint32_t m, uint32_t p, uint32_t j, T &z0, T &z1);

template <>
__device__ __forceinline__ void normal_pair<double>(const NoiseTab &tab, Key key, uint32_t inst, uint32_t tag,
                                                    uint32_t m, uint32_t p, uint32_t j, double &z0,
                                                    double &z1) {
    box_muller(noise_block(key, inst, tag, m, p, j), tab, z0, z1);
}
template <>
__device__ __forceinline__ void normal_pair<float>(const NoiseTab &, Key key, uint32_t inst, uint32_t tag,
                                                   uint32_t m, uint32_t p, uint32_t j, float &z0, float &z1) {
    box_muller_f32(noise_block(key, inst, tag, m, p, j), z0, z1);
}

__device__ __forceinline__ double fmaf_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaf_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// One Euler-Maruyama step of one particle, drift at the old state.
template <int D, typename T>
__device__ __forceinline__ void em_step(T &x, T (&y)[D], const T (&a)[D], const EmCoef<T> &c,
                                        const NoiseTab &tab, Key key, uint32_t inst, uint32_t m, uint32_t p) {
#pragma clang fp contract(off)
    constexpr int NP = (D + 2) / 2;  // pairs of normals for 1 + D components
    T z[2 * NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) normal_pair<T>(tab, key, inst, 0u, m, p, (uint32_t)j, z[2 * j], z[2 * j + 1]);
    T ybar;
    if constexpr (D == 1) {
        ybar = y[0];
    } else {
        T s = (T)0;
#pragma unroll
        for (int i = 0; i < D; ++i) s += y[i];
        ybar = s / (T)D;
    }
    // fused multiply-adds written out, everything else unfused, so that every
    // kernel that inlines this step produces the same bits:
    //   x' = x - dt lam (x - ybar) - dt (c1 + c3 x^2) x + sx z0
    const T d = x - ybar;
    const T x2 = x * x;
    const T cx = fmaf_t(c.a3, x2, c.a1);
    T t = fmaf_t(c.al, d, x);
    t = fmaf_t(cx, x, t);
    const T xn = fmaf_t(c.sx, z[0], t);
    if constexpr (D == 1) {
        // y' = y + (dt/eps) (x - y) + sy z1
        y[0] = fmaf_t(c.sy, z[1], fmaf_t(c.rate, d, y[0]));
    } else {
#pragma unroll
        for (int i = 0; i < D; ++i) y[i] = fmaf_t(c.sy, z[i + 1], fmaf_t(-c.rate, y[i] - a[i] * x, y[i]));
    }
    x = xn;
}

template <typename T>
inline EmCoef<T> make_coef(const pr_sde *s, double dt) {
    EmCoef<T> c;
    c.a3 = (T)(-dt * s->c3);
    c.a1 = (T)(-dt * s->c1);
    c.al = (T)(-dt * s->lambda);
    c.rate = (T)(dt / s->eps);
    c.sx = (T)std::sqrt(2.0 * dt / s->beta);
    c.sy = (T)std::sqrt(2.0 * dt / (s->beta * s->eps));
    return c;
}

}  // namespace pr
