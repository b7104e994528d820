// Chemical-reaction system (Sec. 2.1.2): lognormal initial law, the
// Euler-Maruyama fine propagator with multiplicative noise over all slices
// at once, the mean of the fast variable's equilibrium law and the
// finite-volume coarse propagator with the state-dependent effective
// diffusion (Sec. 2.2.1, the chemical reactions example; Sec. 2.2.2).
//
// Drifts are those of the reaction network whose summed propensities are 2D
// and 2E: b_x = k4 y - k5 x and b_y = k0 - k1 y + k2 y(y-1) - k3 y(y-1)(y-2);
// the diffusions enter the square roots as max(., 0).
#include <algorithm>
#include <cmath>
#include <vector>

#include "pr_chem.hpp"

namespace pr {

struct ChemCoef {
    double ax, ay;                  // dt / tau_x, dt / eps
    double k0, k1, k2, k3, k4, k5;  // reaction rates
};

static ChemCoef make_chem_coef(const pr_chem *c, double dt) {
    ChemCoef k;
    k.ax = dt / c->tau_x;
    k.ay = dt / c->eps;
    k.k0 = c->k[0];
    k.k1 = c->k[1];
    k.k2 = c->k[2];
    k.k3 = c->k[3];
    k.k4 = c->k[4];
    k.k5 = c->k[5];
    return k;
}

// One Euler-Maruyama step of one particle, drift and diffusion at the old
// state (eq. (EMx)/(EMy)).  The Box-Muller radius sqrt(-2 ln u) and the
// noise amplitude sqrt(2 D dt/tau_x) share one square root,
// sqrt(2 D dt/tau_x) z0 = sqrt((2 D dt/tau_x)(-2 ln u)) cos(pi t), and the
// same for Y: two double-precision square roots per step instead of three.
__device__ __forceinline__ void chem_step(double &x, double &y, const ChemCoef &c, const NoiseTab &tab, Key key,
                                          uint32_t inst, uint32_t m, uint32_t p) {
#pragma clang fp contract(off)
    const Block b = noise_block(key, inst, 0u, m, p, 0u);
    // u = (k + 1/2) 2^-52 from the bit fields (exact), L = -2 ln u > 0
    const double u = double_of_words(unit_high_word(b.w0), b.w1) - 0x1.fffffffffffffp-1;
    const double L = neg2_ln(u, tab.lg);
    double sn, cs;
    sincos_cell(b.w2, b.w3, tab.sc, sn, cs);
    const double y1 = y * (y - 1.0);
    const double y2 = y1 * (y - 2.0);
    const double t4 = c.k4 * y;
    const double bx = __builtin_fma(-c.k5, x, t4);  // k4 y - k5 x
    const double d2 = __builtin_fma(c.k5, x, t4);   // 2 D
    const double by = __builtin_fma(-c.k3, y2, __builtin_fma(c.k2, y1, __builtin_fma(-c.k1, y, c.k0)));
    const double e2 = __builtin_fma(c.k3, y2, __builtin_fma(c.k2, y1, __builtin_fma(c.k1, y, c.k0)));  // 2 E
    // a negative D or E is taken as 2^-1000: the amplitude 2^-500 |z| then
    // vanishes in the rounding of x + ... and y + ... like an exact 0
    const double vx = __builtin_fmax(d2 * c.ax * L, 0x1p-1000);
    const double vy = __builtin_fmax(e2 * c.ay * L, 0x1p-1000);
    const double amp_x = sqrt_from_seed(vx, rsq_seed(vx));
    const double amp_y = sqrt_from_seed(vy, rsq_seed(vy));
    x = __builtin_fma(amp_x, cs, __builtin_fma(c.ax, bx, x));
    y = __builtin_fma(amp_y, sn, __builtin_fma(c.ay, by, y));
}

// One thread owns PPT particles of one slice (blockIdx.y) for the whole
// slice; the state stays in registers.
template <int PPT>
__global__ void __launch_bounds__(256) chem_fine_kernel(const double *xin, const double *yin, double *xout,
                                                        double *yout, int64_t n, int slice_first, int64_t S, int N,
                                                        ChemCoef c, Key key, uint32_t inst) {
    __shared__ NoiseTab tab;
    load_noise_tab(tab);
    const int s = blockIdx.y;
    const int sl = slice_first + s;
    const int64_t m0 = uniform_i64(slice_begin(S, N, sl));
    const int64_t m1 = uniform_i64(slice_begin(S, N, sl + 1));
    const int64_t base = (int64_t)blockIdx.x * blockDim.x * PPT + threadIdx.x;
    double xv[PPT], yv[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int64_t p = base + (int64_t)q * blockDim.x;
        const int64_t pc = p < n ? p : 0;
        xv[q] = xin[(int64_t)s * n + pc];
        yv[q] = yin[(int64_t)s * n + pc];
    }
    // 32-bit step counter (the generator's counter word is 32 bits wide)
    const uint32_t mb = (uint32_t)m0, steps = (uint32_t)(m1 - m0);
#pragma unroll 2
    for (uint32_t i = 0; i < steps; ++i) {
#pragma unroll
        for (int q = 0; q < PPT; ++q)
            chem_step(xv[q], yv[q], c, tab, key, inst, mb + i, (uint32_t)(base + (int64_t)q * blockDim.x));
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int64_t p = base + (int64_t)q * blockDim.x;
        if (p >= n) continue;
        xout[(int64_t)s * n + p] = xv[q];
        yout[(int64_t)s * n + p] = yv[q];
    }
}

__global__ void __launch_bounds__(256) chem_init_kernel(double *__restrict__ x, double *__restrict__ y, int64_t n,
                                                        double mx, double sx, double my, double sy, Key key,
                                                        uint32_t inst) {
    __shared__ NoiseTab tab;
    load_noise_tab(tab);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double z0, z1;
    box_muller(noise_block(key, inst, 1u, 0u, (uint32_t)p, 0u), tab, z0, z1);
    x[p] = exp(mx + sx * z0);
    y[p] = exp(my + sy * z1);
}

int check_chem(const pr_chem *c) {
    PR_REQUIRE(c != nullptr, "chem must be non-NULL");
    PR_REQUIRE(c->tau_x > 0.0 && c->eps > 0.0, "need tau_x > 0 and eps > 0");
    for (int i = 0; i < 6; ++i) PR_REQUIRE(c->k[i] >= 0.0 && std::isfinite(c->k[i]), "k%d must be finite and >= 0", i);
    PR_REQUIRE(c->k[4] > 0.0 && c->k[5] > 0.0, "need k4 > 0 and k5 > 0");
    PR_REQUIRE(c->x0_mean > 0.0 && c->y0_mean > 0.0 && c->x0_sd >= 0.0 && c->y0_sd >= 0.0,
               "the lognormal initial law needs means > 0 and sd >= 0");
    return PR_OK;
}

int chem_init_ensemble(const pr_chem *c, uint64_t seed, uint32_t inst, int64_t n, double *x, double *y,
                       hipStream_t st) {
    if (n == 0) return PR_OK;
    const double rx = c->x0_sd / c->x0_mean, ry = c->y0_sd / c->y0_mean;
    const double vx = std::log1p(rx * rx), vy = std::log1p(ry * ry);
    hipLaunchKernelGGL(chem_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, y, n,
                       std::log(c->x0_mean) - 0.5 * vx, std::sqrt(vx), std::log(c->y0_mean) - 0.5 * vy,
                       std::sqrt(vy), make_key(seed), inst);
    PR_LAUNCHED();
    return PR_OK;
}

int chem_fine_propagate(const pr_chem *c, const pr_schedule *sch, uint64_t seed, uint32_t inst, int64_t n,
                        int slice_first, int slice_count, const double *xi, const double *yi, double *x, double *y,
                        hipStream_t st) {
    if (slice_count == 0 || n == 0) return PR_OK;
    constexpr int PPT = 2;
    const dim3 grid((unsigned)((n + 256 * PPT - 1) / (256 * PPT)), (unsigned)slice_count);
    hipLaunchKernelGGL(chem_fine_kernel<PPT>, grid, dim3(256), 0, st, xi, yi, x, y, n, slice_first, sch->total_steps,
                       sch->n_slices, make_chem_coef(c, sch->dt), make_key(seed), inst);
    PR_LAUNCHED();
    return PR_OK;
}

// Trapezoidal rule on y_j = j h, h = 1e-2, j = 0..1e5: running integral of
// b/E from 0, log phi = that - log E, then the normalised first moment.
int chem_mean_fast(const pr_chem *c, double *ybar) {
    constexpr int64_t M = 100000;
    constexpr double h = 1e-2;
    const double *k = c->k;
    std::vector<double> lp(M + 1);
    double run = 0.0, r_prev = 0.0, lmax = -INFINITY;
    for (int64_t j = 0; j <= M; ++j) {
        const double yv = (double)j * h;
        const double y1 = yv * (yv - 1.0), y2 = y1 * (yv - 2.0);
        const double e = 0.5 * (k[0] + k[1] * yv + k[2] * y1 + k[3] * y2);
        PR_REQUIRE(e > 0.0 && std::isfinite(e), "E(y) must stay positive on [0, 1000] (y = %g)", yv);
        const double r = (k[0] - k[1] * yv + k[2] * y1 - k[3] * y2) / e;
        if (j > 0) run += 0.5 * (r_prev + r) * h;
        r_prev = r;
        lp[j] = run - std::log(e);
        lmax = std::max(lmax, lp[j]);
    }
    double z = 0.0, m1 = 0.0;
    for (int64_t j = 0; j <= M; ++j) {
        const double w = (j == 0 || j == M) ? 0.5 * h : h;
        const double phi = std::exp(lp[j] - lmax);
        z += w * phi;
        m1 += w * phi * ((double)j * h);
    }
    *ybar = m1 / z;
    return PR_OK;
}

// Generator of the finite-volume scheme for Fbar'(x) = -(A - k5 x),
// Dbar(x) = (A + k5 x)/2, A = k4 ybar.  With those,
//   log(rho_inf(xa)/rho_inf(xb)) = (4A/k5 - 1) log((A + k5 xa)/(A + k5 xb)) - 2 (xa - xb),
// and each coefficient a_i/g_j = Dbar(x_i)/(tau_x h^2) rho_inf(x_i)/rho_inf(m_j)
// is formed from two neighbouring points.
static int make_chem_generator(const pr_chem *c, double ybar, const pr_grid *grid, std::vector<double> &lo,
                               std::vector<double> &di, std::vector<double> &up) {
    const int I = grid->n_cells;
    const double h = (grid->x_hi - grid->x_lo) / I;
    const double A = c->k[4] * ybar, k5 = c->k[5];
    PR_REQUIRE(A + k5 * grid->x_lo > 0.0, "the effective diffusion must be positive on the grid");
    const double pw = 4.0 * A / k5 - 1.0;
    auto lratio = [&](double xa, double xb) {
        return pw * std::log1p(k5 * (xa - xb) / (A + k5 * xb)) - 2.0 * (xa - xb);
    };
    lo.assign(I, 0.0);
    di.assign(I, 0.0);
    up.assign(I, 0.0);
    for (int i = 1; i < I; ++i) {
        const double e = grid->x_lo + i * h;
        const double ml = grid->x_lo + (i - 0.5) * h, mr = grid->x_lo + (i + 0.5) * h;
        const double base = 0.5 * (A + k5 * e) / (c->tau_x * h * h);
        const double to_left = base * std::exp(lratio(e, ml));   // a_i / g_{i-1}
        const double to_right = base * std::exp(lratio(e, mr));  // a_i / g_i
        di[i - 1] -= to_left;
        lo[i] += to_left;
        di[i] -= to_right;
        up[i - 1] += to_right;
    }
    return PR_OK;
}

int chem_coarse_create(const pr_chem *c, const pr_schedule *sch, const pr_grid *grid, hipStream_t st, Coarse **out) {
    double ybar = 0.0;
    PR_CHECK(chem_mean_fast(c, &ybar));
    std::vector<double> lo, di, up;
    PR_CHECK(make_chem_generator(c, ybar, grid, lo, di, up));
    return coarse_create_tridiag(lo, di, up, sch, grid, st, out);
}

}  // namespace pr

using namespace pr;

extern "C" int pr_chem_init_ensemble(const pr_chem *c, uint64_t seed, uint32_t instance, int64_t n, double *x,
                                     double *y, void *stream) {
    clear_error();
    PR_CHECK(check_chem(c));
    PR_REQUIRE(n >= 0 && n <= 0xFFFFFFFFll, "n must be in [0, 2^32)");
    PR_REQUIRE(n == 0 || (x != nullptr && y != nullptr), "x and y must be non-NULL");
    return chem_init_ensemble(c, seed, instance, n, x, y, as_stream(stream));
}

extern "C" int pr_chem_fine_propagate(const pr_chem *c, const pr_schedule *sched, uint64_t seed, uint32_t instance,
                                      int64_t n, int slice_first, int slice_count, double *x, double *y,
                                      void *stream) {
    clear_error();
    PR_CHECK(check_chem(c));
    PR_CHECK(check_schedule(sched));
    PR_REQUIRE(n >= 0 && n <= 0xFFFFFFFFll, "n must be in [0, 2^32)");
    PR_REQUIRE(slice_first >= 0 && slice_count >= 0 && slice_first + slice_count <= sched->n_slices,
               "slices [%d, %d) outside [0, %d)", slice_first, slice_first + slice_count, sched->n_slices);
    PR_REQUIRE(slice_count <= 65535, "at most 65535 slices per call");
    PR_REQUIRE(n == 0 || slice_count == 0 || (x != nullptr && y != nullptr), "x and y must be non-NULL");
    return chem_fine_propagate(c, sched, seed, instance, n, slice_first, slice_count, x, y, x, y, as_stream(stream));
}

extern "C" int pr_chem_mean_fast(const pr_chem *c, double *ybar) {
    clear_error();
    PR_CHECK(check_chem(c));
    PR_REQUIRE(ybar != nullptr, "ybar must be non-NULL");
    return chem_mean_fast(c, ybar);
}

extern "C" int pr_chem_coarse_create(const pr_chem *c, const pr_schedule *sched, const pr_grid *grid, void *stream,
                                     void **coarse) {
    clear_error();
    PR_CHECK(check_chem(c));
    PR_CHECK(check_schedule(sched));
    PR_CHECK(check_grid(grid));
    PR_REQUIRE(coarse != nullptr, "coarse must be non-NULL");
    Coarse *p = nullptr;
    PR_CHECK(chem_coarse_create(c, sched, grid, as_stream(stream), &p));
    *coarse = p;
    return PR_OK;
}
