// Host harness for the FP64 Box-Muller helpers of the HIP library (the same
// source the kernels inline), used by the CPU tests to compare them with the
// C library and the oracle over many arguments.
#include "pr_normal.hpp"

static pr::NoiseTab host_tab() {
    static const double d[pr::kNoiseTabDoubles] = {
#define PR_NOISE_TABLE_ENTRIES
#include "pr_noise_tables.inc"
#undef PR_NOISE_TABLE_ENTRIES
    };
    pr::NoiseTab t;
    for (int i = 0; i < 256; ++i) t.sc[i] = pr::TabPair{d[2 * i], d[2 * i + 1]};
    for (int i = 0; i < 1024; ++i) t.lg[i] = pr::TabPair{d[512 + 2 * i], d[512 + 2 * i + 1]};
    return t;
}

extern "C" void fm_neg2_ln(const double *u, double *out, long n) {
    const pr::NoiseTab t = host_tab();
    for (long i = 0; i < n; ++i) out[i] = pr::neg2_ln(u[i], t.lg);
}
extern "C" void fm_sqrt_pos(const double *x, double *out, long n) {
    for (long i = 0; i < n; ++i) out[i] = pr::sqrt_pos(x[i]);
}
extern "C" void fm_sqrt_positive(const double *x, double *out, long n) {
    for (long i = 0; i < n; ++i) out[i] = pr::sqrt_positive(x[i]);
}
extern "C" void fm_sincos_cell(const unsigned *w2, const unsigned *w3, double *s, double *c, long n) {
    const pr::NoiseTab t = host_tab();
    for (long i = 0; i < n; ++i) pr::sincos_cell(w2[i], w3[i], t.sc, s[i], c[i]);
}
extern "C" void fm_normal_pair(const unsigned *w, double *z, long n) {
    const pr::NoiseTab t = host_tab();
    for (long i = 0; i < n; ++i)
        pr::normal_pair_of_words(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3], t, z[2 * i], z[2 * i + 1]);
}
