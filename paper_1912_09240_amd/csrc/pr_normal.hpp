// Standard normal pairs from one Philox block (Box-Muller), for the noise of
// the Euler-Maruyama scheme (Sec. 2.1.3 eq. (EMx)/(EMy)) and of the initial
// law.  The random bits are laid out so that both uniforms come out of two
// integer operations:
//
//   u = (k + 1/2) 2^-52,  k = (w0 >> 12) 2^32 + w1            u in (0, 1)
//   t = (i + f) / 128,    i = bits 4..11 of w2,
//                         f = ((w2 >> 12) 2^32 + w3) 2^-52     t in [0, 2)
//   z0 = sqrt(-2 ln u) cos(pi t),  z1 = sqrt(-2 ln u) sin(pi t).
//
// 1 + k 2^-52 and 1 + f are doubles whose high word is 0x3FF00000 | (w >> 12)
// and whose low word is a whole 32-bit word, so each costs one funnel shift.
//
// -2 ln u (table of 1024 pairs, Tang-style reduction):
//   u = m 2^e with m in [1/2, 1); c_i = 1/2 + (i + 1/2)/2048 for the cell i
//   of m (its top 10 mantissa bits), R_i = RN(1/c_i), g = m R_i - 1 with
//   |g| <= 2^-11; -2 ln u = -2 e ln 2 + 2 ln R_i - 2 ln(1 + g), the last term
//   as g (-2 + g - 2g^2/3 + g^3/2 - 2g^4/5) (the next term, g^6/3, is below
//   2^-57 of 2|g|).  The top cell uses R = 1 exactly, so g = m - 1 is exact
//   and -2 ln u keeps full relative accuracy as u -> 1.
// sin and cos of pi t (table of 256 pairs):
//   t = a_i + b/128 with a_i = (i + 1/2)/128 and b = (1 + f) - 3/2 exact in
//   [-1/2, 1/2); with h = pi/128, sin(h b) to b^5 and cos(h b) - 1 to b^6
//   (truncation below 1e-17), then the angle-addition formulas against the
//   tabulated sin(pi a_i), cos(pi a_i).
//
// The tables (pr_noise_tables.inc, written by gen_noise_tables.py) sit in
// LDS during a kernel: every block fills its copy with load_noise_tab()
// before its first normal.  The same code runs on the host against the
// host copy of the tables, for the tests.
#pragma once

#include <cstdint>

#include "pr_fastmath.hpp"

namespace pr {

#include "pr_noise_tables.inc"

struct alignas(16) TabPair {
    double a, b;
};

struct NoiseTab {
    TabPair sc[256];   // sin(pi a_i), cos(pi a_i)
    TabPair lg[1024];  // R_i, 2 ln R_i
};
constexpr int kNoiseTabDoubles = 2560;

static __constant__ double kNoiseTabDev[kNoiseTabDoubles] = {
#define PR_NOISE_TABLE_ENTRIES
#include "pr_noise_tables.inc"
#undef PR_NOISE_TABLE_ENTRIES
};

// 0x3FF00000 | (w >> 12): high word of the double 1 + (w >> 12) 2^-20.
__host__ __device__ __forceinline__ uint32_t unit_high_word(uint32_t w) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_alignbit(0x3FFu, w, 12u);
#else
    return 0x3FF00000u | (w >> 12);
#endif
}

__host__ __device__ __forceinline__ double double_of_words(uint32_t hi, uint32_t lo) {
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// -2 ln u for u in (0, 1); positive for every such u.
__host__ __device__ __forceinline__ double neg2_ln(double u, const TabPair *lg) {
#pragma clang fp contract(off)
    int e;
    const double m = mantissa_exponent(u, e);  // [1/2, 1)
    const uint32_t hi = (uint32_t)(__builtin_bit_cast(uint64_t, m) >> 32);
    const TabPair t = lg[(hi >> 10) & 1023u];
    const double g = __builtin_fma(m, t.a, -1.0);
    double q = __builtin_fma(-0.4, g, 0.5);
    q = __builtin_fma(q, g, -2.0 / 3.0);
    q = __builtin_fma(q, g, 1.0);
    q = __builtin_fma(q, g, -2.0);
    const double s = __builtin_fma(g, q, t.b);  // 2 ln R_i - 2 ln(1 + g)
    return __builtin_fma((double)e, kMinus2Ln2, s);
}

// sin(pi t) -> s, cos(pi t) -> c for t = (i + f)/128 given by words w2, w3.
__host__ __device__ __forceinline__ void sincos_cell(uint32_t w2, uint32_t w3, const TabPair *sc,
                                                     double &s, double &c) {
#pragma clang fp contract(off)
    const TabPair t = sc[(w2 >> 4) & 255u];
    const double b = double_of_words(unit_high_word(w2), w3) - 1.5;
    const double b2 = b * b;
    double ps = __builtin_fma(kSinP5, b2, kSinP3);
    ps = __builtin_fma(ps, b2, kSinP1);
    const double sb = b * ps;  // sin(h b)
    double pc = __builtin_fma(kCosQ6, b2, kCosQ4);
    pc = __builtin_fma(pc, b2, kCosQ2);
    const double cm1 = b2 * pc;  // cos(h b) - 1
    s = __builtin_fma(t.a, cm1, __builtin_fma(t.b, sb, t.a));
    c = __builtin_fma(t.b, cm1, __builtin_fma(-t.a, sb, t.b));
}

// The normal pair of one block of words.
__host__ __device__ __forceinline__ void normal_pair_of_words(uint32_t w0, uint32_t w1, uint32_t w2,
                                                              uint32_t w3, const NoiseTab &tab,
                                                              double &z0, double &z1) {
#pragma clang fp contract(off)
    // 1 + k 2^-52 - (1 - 2^-53) = (k + 1/2) 2^-52, exact
    const double u = double_of_words(unit_high_word(w0), w1) - 0x1.fffffffffffffp-1;
    const double r = sqrt_positive(neg2_ln(u, tab.lg));
    double s, c;
    sincos_cell(w2, w3, tab.sc, s, c);
    z0 = r * c;
    z1 = r * s;
}

// Every thread of the (one-dimensional) block calls this before its first
// normal, and before any early exit.
__device__ __forceinline__ void load_noise_tab(NoiseTab &tab) {
    double *d = reinterpret_cast<double *>(&tab);
    for (int i = (int)threadIdx.x; i < kNoiseTabDoubles; i += (int)blockDim.x) d[i] = kNoiseTabDev[i];
    __syncthreads();
}

}  // namespace pr
