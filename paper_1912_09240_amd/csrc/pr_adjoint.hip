// Pathwise adjoint of the Euler-Maruyama ensemble (d = 1, FP64) with respect
// to theta = (lambda, eps, beta, c3): reverse-mode differentiation of
//   x' = x - dt (c3 x^3 + c1 x + lambda (x - y)) + sx z0,  sx = sqrt(2 dt / beta)
//   y' = y - (dt/eps) (y - x) + sy z1,                     sy = sqrt(2 dt / (beta eps))
// with the noise z held fixed (common random numbers), including the
// dependence of the initial law Y0 = X0 + beta^-1/2 z on beta.
//
// Memory plan: the forward pass stores the state every E steps (E = 256 for
// the differentiated workload; with E <= 8 the checkpoints are the tapes'
// starts and the first recomputation below drops out).
// The reverse kernel walks every particle through the segments backwards.
// For one segment it recomputes the E steps once, writing the state every
// AD_SUB = 8 steps to a small global scratch; then for each 8-step
// sub-segment, last first, it recomputes the 8 states into registers and
// runs the reverse recursion over them.  Every recomputed step is the fine
// propagator's own Euler-Maruyama step (em_step), so the checkpoints and the
// replayed states carry the bits of pr_fine_propagate.  The noise increments
// sx z0, sy z1 of a step are recovered from two consecutive states, so the
// reverse recursion itself needs no random numbers.  Up to four seed vectors
// (observables) are carried at once, giving up to four rows of the Jacobian
// in one sweep.
#include "pr_fine_dev.hpp"
#include "pr_internal.hpp"

namespace pr {

constexpr int AD_SUB = 8;        // steps per register tape
constexpr int AD_THREADS = 128;

struct AdCoef {
    double c3, c1, lam, dt, rate, sx, sy, beta, eps;
};

// One step of the fine propagator (eq. (EMx)/(EMy), d = 1, FP64).
__device__ __forceinline__ void em_step_d1(double &x, double &y, const EmCoef<double> &ec, const NoiseTab &tab,
                                           Key key, uint32_t inst, uint32_t m, uint32_t p) {
    const double a1[1] = {1.0};
    double yv[1] = {y};
    em_step<1, double>(x, yv, a1, ec, tab, key, inst, m, p);
    y = yv[0];
}

// Forward over all steps [0, S) of one segment in time, with checkpoints.
// Two particles per thread (p and p + blockDim), as in the fine propagator,
// so that the two steps' instruction streams interleave.
constexpr int CK_PPT = 2;

__global__ void __launch_bounds__(256) fwd_ckpt_kernel(double *__restrict__ x, double *__restrict__ y, int64_t n,
                                                       int64_t S, int every, double *__restrict__ ckpt,
                                                       EmCoef<double> ec, Key key, uint32_t inst) {
    __shared__ NoiseTab tab;
    load_noise_tab(tab);
    const int64_t base = (int64_t)blockIdx.x * blockDim.x * CK_PPT + threadIdx.x;
    double xv[CK_PPT], yv[CK_PPT];
    bool live[CK_PPT];
    int64_t pp[CK_PPT];
#pragma unroll
    for (int q = 0; q < CK_PPT; ++q) {
        pp[q] = base + (int64_t)q * blockDim.x;
        live[q] = pp[q] < n;
        const int64_t pc = live[q] ? pp[q] : 0;
        xv[q] = x[pc];
        yv[q] = y[pc];
    }
    int64_t cidx = 0;
    for (int64_t m0 = 0; m0 < S; m0 += every, ++cidx) {
#pragma unroll
        for (int q = 0; q < CK_PPT; ++q)
            if (live[q]) {
                ckpt[(cidx * 2) * n + pp[q]] = xv[q];
                ckpt[(cidx * 2 + 1) * n + pp[q]] = yv[q];
            }
        const int64_t m1 = m0 + every < S ? m0 + every : S;
        // 32-bit step counter (the generator's counter word is 32 bits wide)
        const uint32_t mb = (uint32_t)m0, steps = (uint32_t)(m1 - m0);
#pragma unroll 2
        for (uint32_t i = 0; i < steps; ++i) {
#pragma unroll
            for (int q = 0; q < CK_PPT; ++q)
                em_step_d1(xv[q], yv[q], ec, tab, key, inst, mb + i, (uint32_t)pp[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < CK_PPT; ++q)
        if (live[q]) {
            x[pp[q]] = xv[q];
            y[pp[q]] = yv[q];
        }
}

template <int NS>
__global__ void __launch_bounds__(AD_THREADS)
adjoint_kernel(const double *__restrict__ ckpt, int n_ckpt, int every, int64_t n, int64_t S,
               const double *__restrict__ seed_x, const double *__restrict__ seed_y, int from_initial,
               double *__restrict__ sub, double *__restrict__ part, AdCoef c, EmCoef<double> ec, Key key,
               uint32_t inst) {
    __shared__ NoiseTab tab;
    load_noise_tab(tab);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = p < n;
    const int64_t pc = live ? p : 0;
    double ax[NS], ay[NS], g[NS][4];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        ax[k] = live ? seed_x[(int64_t)k * n + pc] : 0.0;
        ay[k] = (live && seed_y) ? seed_y[(int64_t)k * n + pc] : 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) g[k][t] = 0.0;
    }
    const double inv2b = 0.5 / c.beta, inv2e = 0.5 / c.eps, dte2 = c.dt / (c.eps * c.eps);
    if (live) {
        for (int seg = n_ckpt - 1; seg >= 0; --seg) {
            const int64_t m0 = (int64_t)seg * every;
            const int64_t m1 = m0 + every < S ? m0 + every : S;
            // level 1: states every AD_SUB steps of this segment into the
            // scratch; a segment of at most AD_SUB steps is one tape, which
            // starts from the checkpoint itself (checkpoints that close
            // trade memory for this whole recomputation)
            int nsub = 1;
            if (every > AD_SUB) {
                double xv = ckpt[(2 * (int64_t)seg) * n + p], yv = ckpt[(2 * (int64_t)seg + 1) * n + p];
                nsub = 0;
                for (int64_t ms = m0; ms < m1; ms += AD_SUB, ++nsub) {
                    sub[(2 * (int64_t)nsub) * n + p] = xv;
                    sub[(2 * (int64_t)nsub + 1) * n + p] = yv;
                    const int64_t me = ms + AD_SUB < m1 ? ms + AD_SUB : m1;
                    for (int64_t m = ms; m < me; ++m)
                        em_step_d1(xv, yv, ec, tab, key, inst, (uint32_t)m, (uint32_t)p);
                }
            }
            // level 2: each sub-segment, last first; the start of the next
            // one is loaded while this one is replayed
            const double *tj = every > AD_SUB ? sub + (2 * (int64_t)(nsub - 1)) * n : ckpt + (2 * (int64_t)seg) * n;
            double nxs = tj[p], nys = tj[n + p];
            for (int j = nsub - 1; j >= 0; --j) {
                const int64_t ms = m0 + (int64_t)j * AD_SUB;
                const int L = (int)((m1 - ms) < AD_SUB ? (m1 - ms) : AD_SUB);
                double tx[AD_SUB + 1], ty[AD_SUB + 1];
                tx[0] = nxs;
                ty[0] = nys;
                if (j > 0) {  // only with every > AD_SUB (one tape otherwise)
                    nxs = sub[(2 * (int64_t)(j - 1)) * n + p];
                    nys = sub[(2 * (int64_t)(j - 1) + 1) * n + p];
                }
#pragma unroll
                for (int i = 0; i < AD_SUB; ++i) {
                    double a = tx[i], b = ty[i];
                    if (i < L) em_step_d1(a, b, ec, tab, key, inst, (uint32_t)(ms + i), (uint32_t)p);
                    tx[i + 1] = a;
                    ty[i + 1] = b;
                }
#pragma unroll
                for (int i = AD_SUB - 1; i >= 0; --i) {
                    if (i >= L) continue;
                    const double x = tx[i], y = ty[i];
                    const double x2 = x * x;
                    const double fx = c.c3 * x * x * x + c.c1 * x + c.lam * (x - y);
                    const double jxx = 1.0 - c.dt * (3.0 * c.c3 * x2 + c.c1 + c.lam);
                    const double jxy = c.dt * c.lam;
                    const double jyy = 1.0 - c.rate;
                    const double xi_x = tx[i + 1] - x + c.dt * fx;        // sx z0 of this step
                    const double xi_y = ty[i + 1] - y + c.rate * (y - x);  // sy z1 of this step
                    const double dl = -c.dt * (x - y);
                    const double dc3 = -c.dt * x2 * x;
                    const double de = dte2 * (y - x) - inv2e * xi_y;
#pragma unroll
                    for (int k = 0; k < NS; ++k) {
                        g[k][0] += ax[k] * dl;
                        g[k][1] += ay[k] * de;
                        g[k][2] -= inv2b * (ax[k] * xi_x + ay[k] * xi_y);
                        g[k][3] += ax[k] * dc3;
                        const double nax = ax[k] * jxx + ay[k] * c.rate;
                        const double nay = ax[k] * jxy + ay[k] * jyy;
                        ax[k] = nax;
                        ay[k] = nay;
                    }
                }
            }
        }
        if (from_initial) {
            // Y0 = X0 + beta^-1/2 z  =>  dY0/dbeta = -(Y0 - X0) / (2 beta)
            const double dy0 = -(ckpt[n + p] - ckpt[p]) * inv2b;
#pragma unroll
            for (int k = 0; k < NS; ++k) g[k][2] += ay[k] * dy0;
        }
    }
    // block reduction in a fixed order
    __shared__ double red[AD_THREADS / 64][NS * 4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            double v = live ? g[k][t] : 0.0;
            for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) red[wave][k * 4 + t] = v;
        }
    __syncthreads();
    if (threadIdx.x < NS * 4) {
        double v = 0.0;
        for (int w = 0; w < AD_THREADS / 64; ++w) v += red[w][threadIdx.x];
        part[(int64_t)blockIdx.x * NS * 4 + threadIdx.x] = v;
    }
}

__global__ void adjoint_reduce(const double *__restrict__ part, int nblk, int width, double *__restrict__ grad) {
    const int e = blockIdx.x;  // one wave per output element
    const int lane = threadIdx.x;
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += part[(int64_t)b * width + e];
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) grad[e] = s;
}

static AdCoef make_adcoef(const pr_sde *s, double dt) {
    AdCoef c;
    c.c3 = s->c3;
    c.c1 = s->c1;
    c.lam = s->lambda;
    c.dt = dt;
    c.rate = dt / s->eps;
    c.sx = std::sqrt(2.0 * dt / s->beta);
    c.sy = std::sqrt(2.0 * dt / (s->beta * s->eps));
    c.beta = s->beta;
    c.eps = s->eps;
    return c;
}

static int n_checkpoints(int64_t S, int every) { return (int)((S + every - 1) / every); }

size_t adjoint_ws(int64_t n, int every, int n_seed) {
    const int64_t nblk = (n + AD_THREADS - 1) / AD_THREADS;
    const int nsub = (every + AD_SUB - 1) / AD_SUB;
    return sizeof(double) * ((size_t)2 * nsub * n + (size_t)nblk * n_seed * 4) + 512;
}

// Observables of the slow variable and their pathwise seeds (ranks frozen):
// obs[0] = mean x^2, seed 2 x_p / n; obs[1+a] = midpoint (Hazen) quantile at
// alpha_a = (1-f) x_(r) + f x_(r+1), seed (1-f) at particle perm[r], f at
// perm[r+1].  One block.
__global__ void observables_kernel(const double *__restrict__ x, const double *__restrict__ xs,
                                   const uint32_t *__restrict__ perm, const double *__restrict__ mom, int64_t n,
                                   double a0, double a1, double a2, int n_alpha, double *__restrict__ obs,
                                   double *__restrict__ seed) {
#pragma clang fp contract(off)
    const double alpha[3] = {a0, a1, a2};
    if (threadIdx.x == 0) obs[0] = mom[1];
    if (seed) {
        for (int64_t p = threadIdx.x; p < n; p += blockDim.x) seed[p] = 2.0 * x[p] / (double)n;
        for (int a = 0; a < n_alpha; ++a)
            for (int64_t p = threadIdx.x; p < n; p += blockDim.x) seed[(int64_t)(1 + a) * n + p] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x < n_alpha) {
        const int a = threadIdx.x;
        const double t = alpha[a] * (double)n - 0.5;
        double v;
        int64_t r0 = -1, r1 = -1;
        double w0 = 0.0, w1 = 0.0;
        if (t <= 0.0) {
            v = xs[0];
            r0 = 0;
            w0 = 1.0;
        } else if (t >= (double)(n - 1)) {
            v = xs[n - 1];
            r0 = n - 1;
            w0 = 1.0;
        } else {
            const int64_t r = (int64_t)floor(t);
            const double f = t - (double)r;
            v = xs[r] + f * (xs[r + 1] - xs[r]);
            v = v < xs[r + 1] ? v : xs[r + 1];
            r0 = r;
            r1 = r + 1;
            w0 = 1.0 - f;
            w1 = f;
        }
        obs[1 + a] = v;
        if (seed) {
            seed[(int64_t)(1 + a) * n + perm[r0]] = w0;
            if (r1 >= 0) seed[(int64_t)(1 + a) * n + perm[r1]] = w1;
        }
    }
}

size_t observables_ws(int64_t n) {
    return restrict_ws(n, 1, PR_F64) + sizeof(double) * (size_t)n + sizeof(uint32_t) * (size_t)n + 4096;
}

}  // namespace pr

using namespace pr;

extern "C" size_t pr_observables_workspace_size(int64_t n) { return n > 0 ? observables_ws(n) : 4096; }

extern "C" int pr_observables(const double *x, int64_t n, const double *alpha, int n_alpha, double *obs,
                              double *seed_x, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    PR_REQUIRE(n >= 1 && n <= 0xFFFFFFFFll, "n must be in [1, 2^32)");
    PR_REQUIRE(n_alpha >= 0 && n_alpha <= 3, "n_alpha must be in [0, 3]");
    PR_REQUIRE(n_alpha == 0 || alpha != nullptr, "alpha must be non-NULL");
    for (int a = 0; a < n_alpha; ++a) PR_REQUIRE(alpha[a] >= 0.0 && alpha[a] <= 1.0, "alpha must be in [0, 1]");
    PR_REQUIRE(x && obs && ws, "x, obs and ws must be non-NULL");
    if (ws_bytes < observables_ws(n)) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, observables_ws(n));
        return PR_E_NOMEM;
    }
    hipStream_t st = as_stream(stream);
    char *b = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    double *mom = (double *)b;            // 4
    double *q = mom + 4;                  // 2
    double *xs = mom + 8;                 // n
    uint32_t *perm = (uint32_t *)(xs + n);  // n
    void *rws = (void *)(((uintptr_t)(perm + n) + 255) & ~(uintptr_t)255);
    PR_CHECK(restrict_quantiles(x, PR_F64, n, 1, 1, nullptr, q, nullptr, perm, xs, mom, nullptr, rws, st));
    const double a0 = n_alpha > 0 ? alpha[0] : 0.0, a1 = n_alpha > 1 ? alpha[1] : 0.0,
                 a2 = n_alpha > 2 ? alpha[2] : 0.0;
    hipLaunchKernelGGL(observables_kernel, dim3(1), dim3(1024), 0, st, x, (const double *)xs, (const uint32_t *)perm,
                       (const double *)mom, n, a0, a1, a2, n_alpha, obs, seed_x);
    PR_LAUNCHED();
    return PR_OK;
}

static int check_adjoint_sde(const pr_sde *sde) {
    PR_CHECK(check_sde(sde));
    if (sde->d_fast != 1 || sde->precision != PR_F64 || sde->a != nullptr) {
        set_error("the adjoint serves d_fast = 1, FP64, a = NULL");
        return PR_E_UNSUPPORTED;
    }
    return PR_OK;
}

extern "C" int pr_fine_checkpoint(const pr_sde *sde, const pr_schedule *sched, uint64_t seed, uint32_t instance,
                                  int64_t n, void *x, void *y, double *ckpt, int ckpt_every, void *stream) {
    clear_error();
    PR_CHECK(check_adjoint_sde(sde));
    PR_CHECK(check_schedule(sched));
    PR_REQUIRE(n >= 1 && n <= 0xFFFFFFFFll, "n must be in [1, 2^32)");
    PR_REQUIRE(ckpt_every >= 1 && ckpt_every <= 1 << 20, "ckpt_every must be in [1, 2^20]");
    PR_REQUIRE(x && y && ckpt, "x, y and ckpt must be non-NULL");
    hipLaunchKernelGGL(fwd_ckpt_kernel, dim3((unsigned)((n + 256 * CK_PPT - 1) / (256 * CK_PPT))), dim3(256), 0,
                       as_stream(stream),
                       (double *)x, (double *)y, n, sched->total_steps, ckpt_every, ckpt,
                       make_coef<double>(sde, sched->dt), make_key(seed), instance);
    PR_LAUNCHED();
    return PR_OK;
}

extern "C" size_t pr_adjoint_workspace_size(int64_t n, int ckpt_every, int n_seed) {
    if (n <= 0 || ckpt_every <= 0 || n_seed <= 0) return 512;
    return adjoint_ws(n, ckpt_every, n_seed);
}

extern "C" int pr_fine_adjoint(const pr_sde *sde, const pr_schedule *sched, uint64_t seed, uint32_t instance,
                               int64_t n, const double *ckpt, int ckpt_every, const double *seed_x,
                               const double *seed_y, int n_seed, int from_initial, double *grad, void *ws,
                               size_t ws_bytes, void *stream) {
    clear_error();
    PR_CHECK(check_adjoint_sde(sde));
    PR_CHECK(check_schedule(sched));
    PR_REQUIRE(n >= 1 && n <= 0xFFFFFFFFll, "n must be in [1, 2^32)");
    PR_REQUIRE(ckpt_every >= 1 && ckpt_every <= 1 << 20, "ckpt_every must be in [1, 2^20]");
    PR_REQUIRE(n_seed >= 1 && n_seed <= 4, "n_seed must be in [1, 4]");
    PR_REQUIRE(ckpt && seed_x && grad && ws, "ckpt, seed_x, grad and ws must be non-NULL");
    if (ws_bytes < adjoint_ws(n, ckpt_every, n_seed)) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, adjoint_ws(n, ckpt_every, n_seed));
        return PR_E_NOMEM;
    }
    const int nck = n_checkpoints(sched->total_steps, ckpt_every);
    const int64_t nblk = (n + AD_THREADS - 1) / AD_THREADS;
    double *base = (double *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    const int nsub = (ckpt_every + AD_SUB - 1) / AD_SUB;
    double *sub = base;
    double *part = base + (size_t)2 * nsub * n;
    hipStream_t st = as_stream(stream);
    const AdCoef c = make_adcoef(sde, sched->dt);
    const EmCoef<double> ec = make_coef<double>(sde, sched->dt);
    const dim3 grid((unsigned)nblk);
    switch (n_seed) {
        case 1: hipLaunchKernelGGL(adjoint_kernel<1>, grid, dim3(AD_THREADS), 0, st, ckpt, nck, ckpt_every, n,
                                   sched->total_steps, seed_x, seed_y, from_initial, sub, part, c, ec, make_key(seed),
                                   instance); break;
        case 2: hipLaunchKernelGGL(adjoint_kernel<2>, grid, dim3(AD_THREADS), 0, st, ckpt, nck, ckpt_every, n,
                                   sched->total_steps, seed_x, seed_y, from_initial, sub, part, c, ec, make_key(seed),
                                   instance); break;
        case 3: hipLaunchKernelGGL(adjoint_kernel<3>, grid, dim3(AD_THREADS), 0, st, ckpt, nck, ckpt_every, n,
                                   sched->total_steps, seed_x, seed_y, from_initial, sub, part, c, ec, make_key(seed),
                                   instance); break;
        default: hipLaunchKernelGGL(adjoint_kernel<4>, grid, dim3(AD_THREADS), 0, st, ckpt, nck, ckpt_every, n,
                                    sched->total_steps, seed_x, seed_y, from_initial, sub, part, c, ec, make_key(seed),
                                    instance); break;
    }
    PR_LAUNCHED();
    hipLaunchKernelGGL(adjoint_reduce, dim3(n_seed * 4), dim3(64), 0, st, (const double *)part, (int)nblk,
                       n_seed * 4, grad);
    PR_LAUNCHED();
    return PR_OK;
}
