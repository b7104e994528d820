// Fine propagator: initial ensemble and Euler-Maruyama over all slices at once
// (Sec. 2.1.3 eq. (EMx)/(EMy), Sec. 3.2.1).  One thread owns PPT particles of
// one slice and keeps their state in registers for the whole slice; the
// normal increments come from the counter-based generator, so no random
// state is stored and a slice recomputed later sees the same numbers.
#include "pr_fine_dev.hpp"
#include "pr_internal.hpp"

namespace pr {

// With a fast part in R^32 the unrolled FP64 step would take all 256 VGPRs
// (one wave per SIMD); asking for 3 blocks per CU makes the compiler fit it
// in 168 with a few spilled values, which runs 1.5x faster (FP32: 4 blocks,
// 128 VGPRs, 2 % faster than its own 142).
template <int D, typename T, int PPT>
__global__ void __launch_bounds__(256, (D >= 32 ? (sizeof(T) == 4 ? 4 : 3) : 1)) fine_kernel(const T *xin, const T *yin, T *xout, T *yout, int64_t n,
                                                   int slice_first, int64_t S, int N,
                                                   EmCoef<T> c, const double *__restrict__ a_dev,
                                                   Key key, uint32_t inst) {
    __shared__ NoiseTab tab;
    load_noise_tab(tab);
    const int s = blockIdx.y;
    const int sl = slice_first + s;
    // the slice's step range is the block's: keep it in scalar registers so
    // that the step loop's compare runs on the scalar unit
    const int64_t m0 = uniform_i64(slice_begin(S, N, sl));
    const int64_t m1 = uniform_i64(slice_begin(S, N, sl + 1));
    T a[D];
#pragma unroll
    for (int i = 0; i < D; ++i) a[i] = a_dev ? (T)a_dev[i] : (T)1;

    const int64_t base = (int64_t)blockIdx.x * blockDim.x * PPT + threadIdx.x;
    T xv[PPT];
    T yv[PPT][D];
    bool live[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int64_t p = base + (int64_t)q * blockDim.x;
        live[q] = p < n;
        const int64_t pc = live[q] ? p : 0;
        xv[q] = xin[(int64_t)s * n + pc];
#pragma unroll
        for (int i = 0; i < D; ++i) yv[q][i] = yin[((int64_t)s * D + i) * n + pc];
    }
    // 32-bit step counter (the generator's counter word is 32 bits wide);
    // unrolled twice where the registers allow (a large fast part would spill)
    constexpr int UNROLL = D <= 4 ? 2 : 1;
    const uint32_t mb = (uint32_t)m0, steps = (uint32_t)(m1 - m0);
#pragma unroll UNROLL
    for (uint32_t i = 0; i < steps; ++i) {
#pragma unroll
        for (int q = 0; q < PPT; ++q)
            em_step<D, T>(xv[q], yv[q], a, c, tab, key, inst, mb + i, (uint32_t)(base + (int64_t)q * blockDim.x));
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        if (!live[q]) continue;
        const int64_t p = base + (int64_t)q * blockDim.x;
        xout[(int64_t)s * n + p] = xv[q];
#pragma unroll
        for (int i = 0; i < D; ++i) yout[((int64_t)s * D + i) * n + p] = yv[q][i];
    }
}

template <int D, typename T>
__global__ void __launch_bounds__(256) init_kernel(T *__restrict__ x, T *__restrict__ y, int64_t n,
                                                   const double *__restrict__ a_dev, double sd_y,
                                                   Key key, uint32_t inst) {
    __shared__ NoiseTab tab;
    load_noise_tab(tab);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    constexpr int NP = (D + 2) / 2;
    double z[2 * NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) box_muller(noise_block(key, inst, 1u, 0u, (uint32_t)p, (uint32_t)j), tab, z[2 * j], z[2 * j + 1]);
    const double x0 = 0.5 * z[0];
    x[p] = (T)x0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const double ai = a_dev ? a_dev[i] : 1.0;
        y[(int64_t)i * n + p] = (T)(ai * x0 + sd_y * z[i + 1]);
    }
}

__global__ void coupling_kernel(double *a, int d, Key key, uint32_t inst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d) return;
    double u1, u2;
    uniforms53(noise_block(key, inst, 2u, 0u, (uint32_t)i, 0u), u1, u2);
    a[i] = 0.5 + u2;
}

template <int D, typename T>
static int launch_fine(const pr_sde *sde, const pr_schedule *sch, uint64_t seed, uint32_t inst,
                       int64_t n, int slice_first, int slice_count, const void *xi, const void *yi, void *x,
                       void *y, hipStream_t st) {
    constexpr int PPT = (D == 1) ? 2 : 1;
    const int64_t per_block = 256 * PPT;
    dim3 grid((unsigned)((n + per_block - 1) / per_block), (unsigned)slice_count);
    hipLaunchKernelGGL((fine_kernel<D, T, PPT>), grid, dim3(256), 0, st, (const T *)xi, (const T *)yi, (T *)x,
                       (T *)y, n, slice_first,
                       sch->total_steps, sch->n_slices, make_coef<T>(sde, sch->dt), sde->a,
                       make_key(seed), inst);
    PR_LAUNCHED();
    return PR_OK;
}

template <typename T>
static int dispatch_fine(const pr_sde *sde, const pr_schedule *sch, uint64_t seed, uint32_t inst,
                         int64_t n, int sf, int sc, const void *xi, const void *yi, void *x, void *y,
                         hipStream_t st) {
    switch (sde->d_fast) {
        case 1: return launch_fine<1, T>(sde, sch, seed, inst, n, sf, sc, xi, yi, x, y, st);
        case 2: return launch_fine<2, T>(sde, sch, seed, inst, n, sf, sc, xi, yi, x, y, st);
        case 3: return launch_fine<3, T>(sde, sch, seed, inst, n, sf, sc, xi, yi, x, y, st);
        case 4: return launch_fine<4, T>(sde, sch, seed, inst, n, sf, sc, xi, yi, x, y, st);
        case 8: return launch_fine<8, T>(sde, sch, seed, inst, n, sf, sc, xi, yi, x, y, st);
        case 16: return launch_fine<16, T>(sde, sch, seed, inst, n, sf, sc, xi, yi, x, y, st);
        case 32: return launch_fine<32, T>(sde, sch, seed, inst, n, sf, sc, xi, yi, x, y, st);
    }
    set_error("d_fast = %d not served", sde->d_fast);
    return PR_E_UNSUPPORTED;
}

template <int D, typename T>
static int launch_init(const pr_sde *sde, uint64_t seed, uint32_t inst, int64_t n, void *x, void *y,
                       hipStream_t st) {
    dim3 grid((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL((init_kernel<D, T>), grid, dim3(256), 0, st, (T *)x, (T *)y, n, sde->a,
                       1.0 / std::sqrt(sde->beta), make_key(seed), inst);
    PR_LAUNCHED();
    return PR_OK;
}

template <typename T>
static int dispatch_init(const pr_sde *sde, uint64_t seed, uint32_t inst, int64_t n, void *x, void *y,
                         hipStream_t st) {
    switch (sde->d_fast) {
        case 1: return launch_init<1, T>(sde, seed, inst, n, x, y, st);
        case 2: return launch_init<2, T>(sde, seed, inst, n, x, y, st);
        case 3: return launch_init<3, T>(sde, seed, inst, n, x, y, st);
        case 4: return launch_init<4, T>(sde, seed, inst, n, x, y, st);
        case 8: return launch_init<8, T>(sde, seed, inst, n, x, y, st);
        case 16: return launch_init<16, T>(sde, seed, inst, n, x, y, st);
        case 32: return launch_init<32, T>(sde, seed, inst, n, x, y, st);
    }
    set_error("d_fast = %d not served", sde->d_fast);
    return PR_E_UNSUPPORTED;
}

// Host-side entry used by the parareal driver (validation done by caller).
int fine_propagate(const pr_sde *sde, const pr_schedule *sch, uint64_t seed, uint32_t inst, int64_t n,
                   int slice_first, int slice_count, const void *xi, const void *yi, void *x, void *y,
                   hipStream_t st) {
    if (slice_count == 0 || n == 0) return PR_OK;
    if (sde->precision == PR_F64)
        return dispatch_fine<double>(sde, sch, seed, inst, n, slice_first, slice_count, xi, yi, x, y, st);
    return dispatch_fine<float>(sde, sch, seed, inst, n, slice_first, slice_count, xi, yi, x, y, st);
}

int init_ensemble(const pr_sde *sde, uint64_t seed, uint32_t inst, int64_t n, void *x, void *y, hipStream_t st) {
    if (n == 0) return PR_OK;
    if (sde->precision == PR_F64) return dispatch_init<double>(sde, seed, inst, n, x, y, st);
    return dispatch_init<float>(sde, seed, inst, n, x, y, st);
}

}  // namespace pr

using namespace pr;

extern "C" int pr_draw_coupling(uint64_t seed, uint32_t instance, int d, double *a, void *stream) {
    clear_error();
    PR_REQUIRE(d >= 1 && a != nullptr, "need d >= 1 and a != NULL");
    hipLaunchKernelGGL(coupling_kernel, dim3((d + 63) / 64), dim3(64), 0, as_stream(stream), a, d,
                       make_key(seed), instance);
    PR_LAUNCHED();
    return PR_OK;
}

extern "C" int pr_init_ensemble(const pr_sde *sde, uint64_t seed, uint32_t instance, int64_t n,
                                void *x, void *y, void *stream) {
    clear_error();
    PR_CHECK(check_sde(sde));
    PR_REQUIRE(n >= 0 && n <= 0xFFFFFFFFll, "n must be in [0, 2^32)");
    PR_REQUIRE(n == 0 || (x != nullptr && y != nullptr), "x and y must be non-NULL");
    return init_ensemble(sde, seed, instance, n, x, y, as_stream(stream));
}

extern "C" int pr_fine_propagate(const pr_sde *sde, const pr_schedule *sched, uint64_t seed,
                                 uint32_t instance, int64_t n, int slice_first, int slice_count,
                                 void *x, void *y, void *stream) {
    clear_error();
    PR_CHECK(check_sde(sde));
    PR_CHECK(check_schedule(sched));
    PR_REQUIRE(n >= 0 && n <= 0xFFFFFFFFll, "n must be in [0, 2^32)");
    PR_REQUIRE(slice_first >= 0 && slice_count >= 0 && slice_first + slice_count <= sched->n_slices,
               "slices [%d, %d) outside [0, %d)", slice_first, slice_first + slice_count, sched->n_slices);
    PR_REQUIRE(slice_count <= 65535, "at most 65535 slices per call");
    PR_REQUIRE(n == 0 || slice_count == 0 || (x != nullptr && y != nullptr), "x and y must be non-NULL");
    return fine_propagate(sde, sched, seed, instance, n, slice_first, slice_count, x, y, x, y, as_stream(stream));
}
