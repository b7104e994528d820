/*
 * CPU oracle for the micro-macro parareal hot path: particle-level part.
 *
 * TEST INFRASTRUCTURE ONLY.  This file (and everything under oracle/) may be
 * loaded only by the tests, by the smoke check and by the CPU-baseline leg of
 * the benchmark.  The product library never links, loads or calls it, and it
 * shares no code, header or table with the HIP path.
 *
 * Plain scalar C, compiled with -O2 -ffp-contract=off.  Every function states
 * the passage of Legoll, Lelievre, Myerscough and Samaey (arXiv 1912.09240)
 * that it follows.  Where the paper is silent, the reading taken is stated in
 * the comment and listed in the design notes of the repository.
 *
 * Model: the paper's general slow-fast SDE (Sec. 2.1.1, eq. (SDEx)/(SDEy)) with
 * tau_x = 1, D = E = 1/beta, slow potential
 *   F(x, y) = c3 x^4/4 + c1 x^2/2 + lambda (x - ybar)^2/2,  ybar = mean_i y_i,
 * and fast potential G(x, y) = sum_i (y_i - a_i x)^2/2, so that
 *   dX   = -(c3 X^3 + c1 X + lambda (X - mean_i Y_i)) dt + sqrt(2/beta) dW_0
 *   dY_i = -(1/eps)(Y_i - a_i X) dt + sqrt(2/(beta eps)) dW_{i+1}
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int d;          /* fast dimension */
    double lambda;  /* slow-fast coupling */
    double eps;     /* time-scale separation */
    double beta;    /* inverse temperature: D = E = 1/beta */
    double c3;      /* quartic coefficient of the slow potential */
    double c1;      /* quadratic coefficient of the slow potential */
} or_sde;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random numbers: */
/* as easy as 1, 2, 3"): 10 rounds of the 4x32 S-box on a 128-bit counter     */
/* with a 64-bit key bumped by the Weyl constants between rounds.              */
/* ------------------------------------------------------------------------ */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/*
 * Noise stream layout (the paper only asks for independent N(0, dt)
 * increments, Sec. 2.1.3 eq. (EMx)/(EMy), reused across parareal iterations
 * in each slice, Sec. 6).  Reading: one Philox block per (step m, particle p,
 * tag, pair j, instance); key = (lo32(seed), hi32(seed));
 * counter = (m, p, tag << 16 | j, instance).
 * Tags: 0 = Euler-Maruyama increments, 1 = initial condition,
 *       2 = fast-coupling coefficients a_i, 3 = batched-instance parameters.
 */
void or_block(uint64_t seed, uint32_t inst, uint32_t tag, uint32_t m,
              uint32_t p, uint32_t j, uint32_t out[4])
{
    uint32_t ctr[4] = { m, p, (tag << 16) | j, inst };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    or_philox(ctr, key, out);
}

/* Two 53-bit uniforms from one block: u1 in (0,1], u2 in [0,1).  Used for
 * the coupling coefficients; the normals take their bits as below. */
static void or_uniforms(const uint32_t w[4], double *u1, double *u2)
{
    double a = (double)(w[0] >> 5) * 67108864.0 + (double)(w[1] >> 6);
    double b = (double)(w[2] >> 5) * 67108864.0 + (double)(w[3] >> 6);
    *u1 = (a + 0.5) * 0x1p-53;
    *u2 = b * 0x1p-53;
}

/*
 * Box-Muller transform of one block (w0, w1, w2, w3) into two standard
 * normals.  Reading: the paper fixes only the law of the increments, so the
 * bits are laid out for cheap extraction:
 *   u = (k + 1/2) 2^-52,  k = (w0 >> 12) 2^32 + w1          u in (0, 1)
 *   t = (i + f) / 128,    i = (w2 >> 4) mod 256,
 *                         f = ((w2 >> 12) 2^32 + w3) 2^-52   t in [0, 2)
 *   z0 = sqrt(-2 ln u) cos(pi t),  z1 = sqrt(-2 ln u) sin(pi t).
 * u is uniform on a grid of 2^52 midpoints, t on a grid of 2^60 points, so
 * (z0, z1) is the textbook pair of a radius and a uniform angle.
 */
void or_box_muller(const uint32_t w[4], double *z0, double *z1)
{
    uint64_t k = ((uint64_t)(w[0] >> 12) << 32) | w[1];
    uint64_t fbits = ((uint64_t)(w[2] >> 12) << 32) | w[3];
    uint32_t i = (w[2] >> 4) & 255u;
    double u = ((double)k + 0.5) * 0x1p-52;
    double t = ((double)i + (double)fbits * 0x1p-52) / 128.0;
    double r = sqrt(-2.0 * log(u));
    double ang = M_PI * t;
    *z0 = r * cos(ang);
    *z1 = r * sin(ang);
}

/*
 * Normals of the single-precision fine propagator.  Reading: the same block
 * cut to the bits a float carries, the top 24 bits of w0 for the radius and
 * bits 4..31 of w2 for the angle:
 *   u = (k + 1/2) 2^-24,  k = w0 >> 8                         u in (0, 1)
 *   t = (i + f) / 128,    i = (w2 >> 4) mod 256, f = (w2 >> 12) 2^-20
 * and the transform above.  Here u and t are exact and the transform runs in
 * double precision: the law of the variant, without its float rounding.
 */
void or_box_muller_f32(const uint32_t w[4], double *z0, double *z1)
{
    uint32_t k = w[0] >> 8;
    uint32_t i = (w[2] >> 4) & 255u;
    double u = ((double)k + 0.5) * 0x1p-24;
    double t = ((double)i + (double)(w[2] >> 12) * 0x1p-20) / 128.0;
    double r = sqrt(-2.0 * log(u));
    double ang = M_PI * t;
    *z0 = r * cos(ang);
    *z1 = r * sin(ang);
}

/* Normal pair j of (tag, m, p). */
void or_normal_pair(uint64_t seed, uint32_t inst, uint32_t tag, uint32_t m,
                    uint32_t p, uint32_t j, double *z0, double *z1)
{
    uint32_t w[4];
    or_block(seed, inst, tag, m, p, j, w);
    or_box_muller(w, z0, z1);
}

/* The same pair with the single-precision variant's normals. */
static void or_normal_pair_f32(uint64_t seed, uint32_t inst, uint32_t tag, uint32_t m,
                               uint32_t p, uint32_t j, double *z0, double *z1)
{
    uint32_t w[4];
    or_block(seed, inst, tag, m, p, j, w);
    or_box_muller_f32(w, z0, z1);
}

/* Normal number `idx` of (tag, m, p): index 2j is z0 of pair j, 2j+1 is z1. */
static double or_normal(uint64_t seed, uint32_t inst, uint32_t tag, uint32_t m,
                        uint32_t p, int idx)
{
    double z0, z1;
    or_normal_pair(seed, inst, tag, m, p, (uint32_t)(idx / 2), &z0, &z1);
    return (idx % 2 == 0) ? z0 : z1;
}

/* Array form for tests: out[p][k] = normal k of particle p0+p, k < n_norm. */
void or_normals(uint64_t seed, uint32_t inst, uint32_t tag, uint32_t m,
                int64_t p0, int64_t n, int n_norm, double *out)
{
    for (int64_t p = 0; p < n; ++p)
        for (int k = 0; k < n_norm; ++k)
            out[p * n_norm + k] = or_normal(seed, inst, tag, m, (uint32_t)(p0 + p), k);
}

/* Raw blocks for tests: out[p][4]. */
void or_blocks(uint64_t seed, uint32_t inst, uint32_t tag, uint32_t m,
               int64_t p0, int64_t n, uint32_t j, uint32_t *out)
{
    for (int64_t p = 0; p < n; ++p)
        or_block(seed, inst, tag, m, (uint32_t)(p0 + p), j, out + 4 * p);
}

/* ------------------------------------------------------------------------ */
/* Fast coupling coefficients a_i ~ U(0.5, 1.5) (d > 1 workloads): reading,  */
/* a_i = 0.5 + u2 of the block (tag 2, m = 0, p = i, j = 0).                 */
/* ------------------------------------------------------------------------ */
void or_coupling(uint64_t seed, uint32_t inst, int d, double *a)
{
    for (int i = 0; i < d; ++i) {
        uint32_t w[4];
        double u1, u2;
        or_block(seed, inst, 2u, 0u, (uint32_t)i, 0u, w);
        or_uniforms(w, &u1, &u2);
        a[i] = 0.5 + u2;
    }
}

/* ------------------------------------------------------------------------ */
/* Batched-instance parameters (one block, tag 3, m = p = j = 0), four      */
/* 32-bit uniforms u_k = (w_k + 1/2) 2^-32:                                  */
/*   eps = 10^(-3 + 2 u0), lambda = 0.5 + 1.5 u1,                            */
/*   log2 N = 12 + floor(7 u2), slices = 8 + floor(57 u3).                   */
/* ------------------------------------------------------------------------ */
void or_instance_params(uint64_t seed, uint32_t inst, double *eps, double *lambda,
                        int64_t *n, int *n_slices)
{
    uint32_t w[4];
    double u[4];
    or_block(seed, inst, 3u, 0u, 0u, 0u, w);
    for (int k = 0; k < 4; ++k) u[k] = ((double)w[k] + 0.5) * 0x1p-32;
    *eps = pow(10.0, -3.0 + 2.0 * u[0]);
    *lambda = 0.5 + 1.5 * u[1];
    *n = (int64_t)1 << (12 + (int)floor(7.0 * u[2]));
    *n_slices = 8 + (int)floor(57.0 * u[3]);
}

/* ------------------------------------------------------------------------ */
/* Initial ensemble (the paper leaves X0, Y0 to the experiment, Sec. 2.1.1). */
/* Reading: X0 ~ N(0, 0.25) (variance), Y0_i ~ N(a_i X0, 1/beta), from the   */
/* normals of tag 1 at m = 0: normal 0 -> X0, normal i+1 -> Y0_i.            */
/* y is stored [d][n].                                                       */
/* ------------------------------------------------------------------------ */
void or_init_ensemble(const or_sde *s, const double *a, uint64_t seed, uint32_t inst,
                      int64_t n, double *x, double *y)
{
    double sd_y = 1.0 / sqrt(s->beta);
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        double x0 = 0.5 * or_normal(seed, inst, 1u, 0u, (uint32_t)p, 0);
        x[p] = x0;
        for (int i = 0; i < s->d; ++i) {
            double ai = a ? a[i] : 1.0;
            y[(int64_t)i * n + p] = ai * x0 + sd_y * or_normal(seed, inst, 1u, 0u, (uint32_t)p, i + 1);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Euler-Maruyama (Sec. 2.1.3, eq. (EMx)/(EMy)): drift at the old state,     */
/* increments sqrt(dt) z with z from the noise layout above (tag 0, m = the  */
/* global step index).  Advances particles [p0, p0+n) over global steps      */
/* [m_begin, m_end).  x[n], y[d][n] in place.  f32_noise selects the normals */
/* of the single-precision propagator (the scheme itself stays in double).   */
/* ------------------------------------------------------------------------ */
static void em_propagate(const or_sde *s, const double *a, uint64_t seed, uint32_t inst,
                         int64_t p0, int64_t n, int64_t m_begin, int64_t m_end,
                         double dt, double *x, double *y, int f32_noise)
{
    int d = s->d;
    double sx = sqrt(2.0 * dt / s->beta);
    double sy = sqrt(2.0 * dt / (s->beta * s->eps));
    double rate = dt / s->eps;
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        double *z = (double *)malloc(sizeof(double) * (size_t)(d + 2));
        double *yv = (double *)malloc(sizeof(double) * (size_t)d);
        uint32_t p = (uint32_t)(p0 + q);
        double xv = x[q];
        for (int i = 0; i < d; ++i) yv[i] = y[(int64_t)i * n + q];
        for (int64_t m = m_begin; m < m_end; ++m) {
            for (int k = 0; k < d + 1; k += 2) {
                if (f32_noise)
                    or_normal_pair_f32(seed, inst, 0u, (uint32_t)m, p, (uint32_t)(k / 2), &z[k], &z[k + 1]);
                else
                    or_normal_pair(seed, inst, 0u, (uint32_t)m, p, (uint32_t)(k / 2), &z[k], &z[k + 1]);
            }
            double ybar = 0.0;
            for (int i = 0; i < d; ++i) ybar += yv[i];
            ybar = ybar / (double)d;
            double fx = s->c3 * xv * xv * xv + s->c1 * xv + s->lambda * (xv - ybar);
            double xn = xv - dt * fx + sx * z[0];
            for (int i = 0; i < d; ++i) {
                double ai = a ? a[i] : 1.0;
                yv[i] = yv[i] - rate * (yv[i] - ai * xv) + sy * z[i + 1];
            }
            xv = xn;
        }
        x[q] = xv;
        for (int i = 0; i < d; ++i) y[(int64_t)i * n + q] = yv[i];
        free(z);
        free(yv);
    }
}

void or_em_propagate(const or_sde *s, const double *a, uint64_t seed, uint32_t inst,
                     int64_t p0, int64_t n, int64_t m_begin, int64_t m_end,
                     double dt, double *x, double *y)
{
    em_propagate(s, a, seed, inst, p0, n, m_begin, m_end, dt, x, y, 0);
}

void or_em_propagate_f32noise(const or_sde *s, const double *a, uint64_t seed, uint32_t inst,
                              int64_t p0, int64_t n, int64_t m_begin, int64_t m_end,
                              double dt, double *x, double *y)
{
    em_propagate(s, a, seed, inst, p0, n, m_begin, m_end, dt, x, y, 1);
}

/* ------------------------------------------------------------------------ */
/* Pathwise tangents (forward mode) of the Euler-Maruyama ensemble with      */
/* respect to theta = (lambda, eps, beta, c3), for d = 1 and a = 1, starting */
/* from the initial ensemble (whose Y0 depends on beta through its standard  */
/* deviation).  Noise is held fixed (common random numbers).  On return      */
/* x[n], y[n] hold the state at step m_end and dx[4][n], dy[4][n] its        */
/* derivatives.                                                              */
/* ------------------------------------------------------------------------ */
void or_em_tangent(const or_sde *s, uint64_t seed, uint32_t inst, int64_t n,
                   int64_t m_end, double dt, double *x, double *y, double *dx, double *dy)
{
    double beta = s->beta, eps = s->eps, lam = s->lambda, c3 = s->c3, c1 = s->c1;
    double sx = sqrt(2.0 * dt / beta);
    double sy = sqrt(2.0 * dt / (beta * eps));
    double rate = dt / eps;
    /* d sx / d theta and d sy / d theta */
    double dsx[4] = { 0.0, 0.0, -0.5 * sx / beta, 0.0 };
    double dsy[4] = { 0.0, -0.5 * sy / eps, -0.5 * sy / beta, 0.0 };
    double drate[4] = { 0.0, -dt / (eps * eps), 0.0, 0.0 };
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        double z0, z1;
        or_normal_pair(seed, inst, 1u, 0u, (uint32_t)p, 0u, &z0, &z1);
        double sd_y = 1.0 / sqrt(beta);
        double xv = 0.5 * z0;
        double yv = 1.0 * xv + sd_y * z1;
        double tx[4] = { 0.0, 0.0, 0.0, 0.0 };
        double ty[4] = { 0.0, 0.0, -0.5 * z1 / (beta * sqrt(beta)), 0.0 };
        for (int64_t m = 0; m < m_end; ++m) {
            or_normal_pair(seed, inst, 0u, (uint32_t)m, (uint32_t)p, 0u, &z0, &z1);
            double fx = c3 * xv * xv * xv + c1 * xv + lam * (xv - yv);
            double dfx_dx = 3.0 * c3 * xv * xv + c1 + lam;
            double dfx_dy = -lam;
            /* explicit theta dependence of fx: lambda -> (x - y), c3 -> x^3 */
            double pfx[4] = { xv - yv, 0.0, 0.0, xv * xv * xv };
            double gy = yv - xv; /* fast drift is -(1/eps) gy */
            double ntx[4], nty[4];
            for (int k = 0; k < 4; ++k) {
                ntx[k] = tx[k] - dt * (dfx_dx * tx[k] + dfx_dy * ty[k] + pfx[k]) + dsx[k] * z0;
                nty[k] = ty[k] - rate * (ty[k] - tx[k]) - drate[k] * gy + dsy[k] * z1;
            }
            double xn = xv - dt * fx + sx * z0;
            double yn = yv - rate * gy + sy * z1;
            xv = xn;
            yv = yn;
            for (int k = 0; k < 4; ++k) { tx[k] = ntx[k]; ty[k] = nty[k]; }
        }
        x[p] = xv;
        y[p] = yv;
        for (int k = 0; k < 4; ++k) {
            dx[(int64_t)k * n + p] = tx[k];
            dy[(int64_t)k * n + p] = ty[k];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Chemical-reaction system (Sec. 2.1.2): slow X, fast Y, multiplicative      */
/* noise.  The SDE is eq. (SDEx)/(SDEy) with the diffusions                   */
/*   D(x, y) = (k4 y + k5 x)/2,                                               */
/*   E(y)    = (k0 + k1 y + k2 y(y-1) + k3 y(y-1)(y-2))/2,                    */
/* which are half the summed propensities of the reactions                    */
/*   0 -> Y (k0), Y -> 0 (k1 y), 2Y -> 3Y (k2 y(y-1)), 3Y -> 2Y               */
/*   (k3 y(y-1)(y-2)), Y -> Y + X (k4 y), X -> 0 (k5 x).                      */
/* Reading of the potentials: the drifts are the chemical-Langevin drifts of  */
/* those reactions,                                                           */
/*   -dF/dx = k4 y - k5 x,                                                    */
/*   -dG/dy = k0 - k1 y + k2 y(y-1) - k3 y(y-1)(y-2),                         */
/* i.e. F = -k4 x y + k5 x^2/2 and                                            */
/* G = -k0 y + k1 y^2/2 - k2 y^2 (y/3 - 1/2) + k3 y^2 (y/2 - 1)^2.  The signs  */
/* printed for the k1, k2, k3 and k5 terms give drifts without a stable state  */
/* (X and Y grow without bound), which contradicts the bounded grid and the   */
/* bistability of the fast variable that the experiments rely on.            */
/* Reading of D >= 0: the diffusions enter the square root as max(., 0).      */
/* ------------------------------------------------------------------------ */
typedef struct {
    double tau_x;     /* slow time scale */
    double eps;       /* time-scale separation */
    double k[6];      /* reaction rates k0..k5 */
    double x0_mean, x0_sd, y0_mean, y0_sd;  /* lognormal initial law */
} or_chem;

/* Initial law (Sec. 6): independent lognormal X0, Y0 with the given mean and
 * standard deviation: log X0 ~ N(mu, s^2), s^2 = log(1 + (sd/mean)^2),
 * mu = log(mean) - s^2/2.  X0 from normal 0, Y0 from normal 1 of the pair
 * (tag 1, m = 0, p, j = 0). */
void or_chem_init(const or_chem *c, uint64_t seed, uint32_t inst, int64_t n, double *x, double *y)
{
    double vx = log(1.0 + (c->x0_sd / c->x0_mean) * (c->x0_sd / c->x0_mean));
    double vy = log(1.0 + (c->y0_sd / c->y0_mean) * (c->y0_sd / c->y0_mean));
    double mx = log(c->x0_mean) - 0.5 * vx, my = log(c->y0_mean) - 0.5 * vy;
    double sx = sqrt(vx), sy = sqrt(vy);
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        double z0, z1;
        or_normal_pair(seed, inst, 1u, 0u, (uint32_t)p, 0u, &z0, &z1);
        x[p] = exp(mx + sx * z0);
        y[p] = exp(my + sy * z1);
    }
}

/* Euler-Maruyama (Sec. 2.1.3 eq. (EMx)/(EMy)) for the system above, drift and
 * diffusion at the old state, normals (z0, z1) of pair (tag 0, m, p, j = 0):
 *   X' = X + (dt/tau_x)(k4 Y - k5 X) + sqrt(2 max(D, 0) dt/tau_x) z0
 *   Y' = Y + (dt/eps) b(Y)          + sqrt(2 max(E, 0) dt/eps) z1
 * for global steps [m_begin, m_end) of particles p0 .. p0+n-1. */
void or_chem_em(const or_chem *c, uint64_t seed, uint32_t inst, int64_t p0, int64_t n, int64_t m_begin,
                int64_t m_end, double dt, double *x, double *y)
{
    const double *k = c->k;
    double ax = dt / c->tau_x, ay = dt / c->eps;
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        uint32_t p = (uint32_t)(p0 + q);
        double xv = x[q], yv = y[q];
        for (int64_t m = m_begin; m < m_end; ++m) {
            double z0, z1;
            or_normal_pair(seed, inst, 0u, (uint32_t)m, p, 0u, &z0, &z1);
            double y1 = yv * (yv - 1.0);
            double y2 = y1 * (yv - 2.0);
            double bx = k[4] * yv - k[5] * xv;
            double by = k[0] - k[1] * yv + k[2] * y1 - k[3] * y2;
            double D = 0.5 * (k[4] * yv + k[5] * xv);
            double E = 0.5 * (k[0] + k[1] * yv + k[2] * y1 + k[3] * y2);
            if (D < 0.0) D = 0.0;
            if (E < 0.0) E = 0.0;
            double xn = xv + ax * bx + sqrt(2.0 * D * ax) * z0;
            double yn = yv + ay * by + sqrt(2.0 * E * ay) * z1;
            xv = xn;
            yv = yn;
        }
        x[q] = xv;
        y[q] = yv;
    }
}
