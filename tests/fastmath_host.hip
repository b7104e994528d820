// Host harness for the FP64 Box-Muller helpers of the HIP library, used by the
// CPU tests to compare them with the C library over many arguments.
#include "pr_fastmath.hpp"

extern "C" void fm_log_unit(const double *u, double *out, long n) {
    for (long i = 0; i < n; ++i) out[i] = pr::log_unit(u[i]);
}
extern "C" void fm_sqrt_pos(const double *x, double *out, long n) {
    for (long i = 0; i < n; ++i) out[i] = pr::sqrt_pos(x[i]);
}
extern "C" void fm_sincos_half_turn(const double *t, double *s, double *c, long n) {
    for (long i = 0; i < n; ++i) pr::sincos_half_turn(t[i], s[i], c[i]);
}
