// Coarse propagator (Sec. 2.2): finite volumes for the slow Fokker-Planck
// equation in the rho/rho_inf form with central differences on a uniform
// grid, advanced by the exact exponential E(tau) = exp(A tau) (Sec. 2.2.2),
// plus the conversions between quantile knots and cell masses through the
// piecewise-linear cdf (Sec. 4.4, eq. (discr_cdf)) and the quantile iterator
// with its monotone repair.
//
// A is tridiagonal; E(tau) is dense.  It is built once per distinct slice
// length on the device by scaling and squaring: X = A tau / 2^s with
// ||X||_1 <= 1, a degree-24 Taylor polynomial by Horner's rule, then s
// squarings, all with an LDS-tiled FP64 GEMM.  Applying E is a batched
// matrix-vector product (FP64 VALU; the matrix stays in L2/MALL).
#include <cmath>
#include <vector>

#include "pr_chem.hpp"
#include "pr_coarse_dev.hpp"
#include "pr_internal.hpp"

namespace pr {

// ---------------------------------------------------------------------------
// FP64 GEMM C = alpha * A B + diag * I (n x n, row-major), 64x64 tiles.
// ---------------------------------------------------------------------------
constexpr int GM_T = 64, GM_K = 16;

__global__ void __launch_bounds__(256) gemm_f64(const double *__restrict__ A, const double *__restrict__ B,
                                                double *__restrict__ C, int n, double alpha, double diag) {
    __shared__ double As[GM_K][GM_T + 1];
    __shared__ double Bs[GM_K][GM_T + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int row0 = blockIdx.y * GM_T, col0 = blockIdx.x * GM_T;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < n; k0 += GM_K) {
        for (int e = threadIdx.x; e < GM_T * GM_K; e += 256) {
            const int r = e / GM_K, c = e % GM_K;  // A tile: rows row0+r, cols k0+c
            const int gr = row0 + r, gc = k0 + c;
            As[c][r] = (gr < n && gc < n) ? A[(int64_t)gr * n + gc] : 0.0;
            const int br = e / GM_T, bc = e % GM_T;  // B tile: rows k0+br, cols col0+bc
            const int gbr = k0 + br, gbc = col0 + bc;
            Bs[br][bc] = (gbr < n && gbc < n) ? B[(int64_t)gbr * n + gbc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GM_K; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = row0 + ty + 16 * i, c = col0 + tx + 16 * j;
            if (r < n && c < n) C[(int64_t)r * n + c] = alpha * acc[i][j] + (r == c ? diag : 0.0);
        }
}

// X = A_tridiag * scale, dense.
__global__ void tridiag_to_dense(const double *__restrict__ lo, const double *__restrict__ di,
                                 const double *__restrict__ up, int n, double scale, double *__restrict__ X,
                                 double add_identity_over) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int r = (int)(e / n), c = (int)(e % n);
    double v = 0.0;
    if (c == r) v = di[r] * scale;
    else if (c == r + 1) v = up[r] * scale;
    else if (c == r - 1) v = lo[r] * scale;
    if (add_identity_over != 0.0) v = v * add_identity_over + (r == c ? 1.0 : 0.0);
    X[e] = v;
}

__global__ void __launch_bounds__(256) knots_to_masses(const double *__restrict__ q, int q_stride,
                                                       double *__restrict__ rho, GridDev g) {
#pragma clang fp contract(off)
    extern __shared__ double sh[];
    double *qs = sh;               // nq + 1
    double *c = sh + g.nq + 1;     // cells + 1 (edges 1..cells-1 used)
    const int s = blockIdx.x;
    for (int j = threadIdx.x; j <= g.nq; j += blockDim.x) qs[j] = q[(int64_t)s * q_stride + j];
    __syncthreads();
    for (int i = 1 + threadIdx.x; i < g.cells; i += blockDim.x) c[i] = cdf_knots(qs, g.nq, edge_at(g, i));
    __syncthreads();
    double *r = rho + (int64_t)s * g.cells;
    for (int i = threadIdx.x; i < g.cells; i += blockDim.x) {
        double v;
        if (i == 0) v = c[1];
        else if (i == g.cells - 1) v = 1.0 - c[g.cells - 1];
        else v = c[i + 1] - c[i];
        r[i] = v;
    }
}

// One chain link's coarse step without the masses in global memory: every
// block turns the knots q into the cell masses (the arithmetic of
// knots_to_masses) in LDS and forms its four rows of max(E rho, 0).
__global__ void __launch_bounds__(256) apply_expm_knots(const double *__restrict__ E, const int *__restrict__ tau_id,
                                                        int slice, const double *__restrict__ q,
                                                        double *__restrict__ rout, GridDev g) {
#pragma clang fp contract(off)
    extern __shared__ double sh[];
    const int n = g.cells;
    double *qs = sh;            // nq + 1
    double *c = qs + g.nq + 1;  // cells + 1
    double *rv = c + n + 1;     // cells
    for (int j = threadIdx.x; j <= g.nq; j += blockDim.x) qs[j] = q[j];
    __syncthreads();
    for (int i = 1 + threadIdx.x; i < n; i += blockDim.x) c[i] = cdf_knots(qs, g.nq, edge_at(g, i));
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        rv[i] = (i == 0) ? c[1] : (i == n - 1) ? 1.0 - c[n - 1] : c[i + 1] - c[i];
    __syncthreads();
    const double *Es = E + (int64_t)tau_id[slice] * n * n;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + wave;
    if (r >= n) return;
    const double *row = Es + (int64_t)r * n;
    double acc = lane_row_dot(row, rv, n, lane);
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) rout[r] = acc > 0.0 ? acc : 0.0;
}

// rho_out[s] = max(E_{id(s)} rho_in[s], 0).  One wave per row.
__global__ void __launch_bounds__(256) apply_expm(const double *__restrict__ E, const int *__restrict__ tau_id,
                                                  int slice_first, const double *__restrict__ rin,
                                                  double *__restrict__ rout, int n) {
    extern __shared__ double rv[];
    const int s = blockIdx.y;
    const double *Es = E + (int64_t)tau_id[slice_first + s] * n * n;
    for (int j = threadIdx.x; j < n; j += blockDim.x) rv[j] = rin[(int64_t)s * n + j];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + wave;
    if (r >= n) return;
    const double *row = Es + (int64_t)r * n;
    double acc = lane_row_dot(row, rv, n, lane);
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) rout[(int64_t)s * n + r] = acc > 0.0 ? acc : 0.0;
}

__global__ void __launch_bounds__(256) masses_to_knots(const double *__restrict__ rho, double *__restrict__ q,
                                                       int q_stride, GridDev g) {
    extern __shared__ double sh[];
    double *r = sh;
    double *C = sh + g.cells;
    const int s = blockIdx.x;
    for (int i = threadIdx.x; i < g.cells; i += blockDim.x) r[i] = rho[(int64_t)s * g.cells + i];
    __syncthreads();
    masses_to_knots_block(r, C, g, q + (int64_t)s * q_stride);
}

// Quantile iterator on fixed levels: q_new = PAVA(q_f + (q_c_next - q_c_star)).
// Fused with the Qf of the coarse result: rho is C applied to q_new^n.
__global__ void __launch_bounds__(256) qf_and_jump(const double *__restrict__ rho, const double *__restrict__ qf,
                                                   const double *__restrict__ qcs, double *__restrict__ q_out,
                                                   double *__restrict__ qc_out, GridDev g) {
#pragma clang fp contract(off)
    extern __shared__ double sh[];
    double *r = sh;
    double *C = r + g.cells;
    double *qc = C + g.cells + 1;
    double *S = qc + g.nq + 1;
    int *SC = (int *)(S + g.nq + 1);
    int *vio = SC + g.nq + 1;
    for (int i = threadIdx.x; i < g.cells; i += blockDim.x) r[i] = rho[i];
    __syncthreads();
    masses_to_knots_block(r, C, g, qc);
    __syncthreads();
    for (int j = threadIdx.x; j <= g.nq; j += blockDim.x) {
        if (qc_out) qc_out[j] = qc[j];
        qc[j] = qf[j] + (qc[j] - qcs[j]);
    }
    __syncthreads();
    pava_block(qc, g.nq + 1, S, SC, vio);
    for (int j = threadIdx.x; j <= g.nq; j += blockDim.x) q_out[j] = qc[j];
}

// The quantile iterator alone on k independent rows of L = Q + 1 knots:
// q_out[s] = PAVA(q_f[s] + (q_c_next[s] - q_c_star[s])), the arithmetic and the
// monotone repair of qf_and_jump.  One block per row; every row is read into
// LDS before any write, so q_out may alias the inputs row for row.
__global__ void __launch_bounds__(256) quantile_jump_rows(const double *__restrict__ qcn, const double *__restrict__ qf,
                                                          const double *__restrict__ qcs, double *q_out, int L) {
#pragma clang fp contract(off)
    extern __shared__ double sh[];
    double *qc = sh;
    double *S = qc + L;
    int *SC = (int *)(S + L);
    int *vio = SC + L;
    const int64_t o = (int64_t)blockIdx.x * L;
    for (int j = threadIdx.x; j < L; j += blockDim.x) qc[j] = qf[o + j] + (qcn[o + j] - qcs[o + j]);
    __syncthreads();
    pava_block(qc, L, S, SC, vio);
    for (int j = threadIdx.x; j < L; j += blockDim.x) q_out[o + j] = qc[j];
}

// ---------------------------------------------------------------------------
// Handle.
// ---------------------------------------------------------------------------
struct Coarse {
    GridDev g;
    int n_slices;
    int n_tau;
    double *E = nullptr;    // [n_tau][I][I]
    int *tau_id = nullptr;  // [n_slices]
    double *rho_a = nullptr, *rho_b = nullptr;  // [n_slices][I] scratch
    std::vector<double> taus;
    int device = 0;
};

int build_expm(const std::vector<double> &lo, const std::vector<double> &di, const std::vector<double> &up,
                      int n, double tau, double *out, double *w1, double *w2, double *w3, hipStream_t st) {
    // ||A tau||_1 = max column sum of |entries|
    double norm = 0.0;
    for (int c = 0; c < n; ++c) {
        double s = std::fabs(di[c]);
        if (c > 0) s += std::fabs(up[c - 1]);
        if (c + 1 < n) s += std::fabs(lo[c + 1]);
        norm = std::max(norm, s * tau);
    }
    int sq = 0;
    while (norm / std::ldexp(1.0, sq) > 1.0) ++sq;
    const double scale = tau / std::ldexp(1.0, sq);
    constexpr int M = 24;  // ||X|| <= 1: truncation below 1/25! ~ 6e-26
    double *d_lo, *d_di, *d_up;
    PR_HIP(hipMalloc(&d_lo, sizeof(double) * n * 3));
    d_di = d_lo + n;
    d_up = d_lo + 2 * n;
    PR_HIP(hipMemcpyAsync(d_lo, lo.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    PR_HIP(hipMemcpyAsync(d_di, di.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    PR_HIP(hipMemcpyAsync(d_up, up.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    const int64_t nn = (int64_t)n * n;
    const dim3 eg((unsigned)((nn + 255) / 256));
    // X = A tau / 2^s into w1; R = I + X / M into w2
    hipLaunchKernelGGL(tridiag_to_dense, eg, dim3(256), 0, st, d_lo, d_di, d_up, n, scale, w1, 0.0);
    hipLaunchKernelGGL(tridiag_to_dense, eg, dim3(256), 0, st, d_lo, d_di, d_up, n, scale, w2, 1.0 / M);
    PR_LAUNCHED();
    const dim3 gg((n + GM_T - 1) / GM_T, (n + GM_T - 1) / GM_T);
    double *R = w2, *T = w3;
    for (int k = M - 1; k >= 1; --k) {  // R = I + X R / k
        hipLaunchKernelGGL(gemm_f64, gg, dim3(256), 0, st, (const double *)w1, (const double *)R, T, n, 1.0 / k, 1.0);
        PR_LAUNCHED();
        std::swap(R, T);
    }
    for (int i = 0; i < sq; ++i) {
        double *dst = (i == sq - 1) ? out : T;
        hipLaunchKernelGGL(gemm_f64, gg, dim3(256), 0, st, (const double *)R, (const double *)R, dst, n, 1.0, 0.0);
        PR_LAUNCHED();
        if (dst == T) std::swap(R, T);
    }
    if (sq == 0) PR_HIP(hipMemcpyAsync(out, R, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
    PR_HIP(hipStreamSynchronize(st));
    PR_HIP(hipFree(d_lo));
    return PR_OK;
}

// Tridiagonal generator of the finite-volume scheme: lo[i] = A[i][i-1],
// di[i] = A[i][i], up[i] = A[i][i+1].
int make_generator(const pr_sde *sde, const pr_grid *grid, std::vector<double> &lo, std::vector<double> &di,
                   std::vector<double> &up, hipStream_t st) {
    const int I = grid->n_cells;
    const double h = (grid->x_hi - grid->x_lo) / I;
    // effective potential V = c3 x^4/4 + k2 x^2/2, k2 = c1 + lambda (1 - mean a)
    double abar = 1.0;
    if (sde->a) {
        std::vector<double> a(sde->d_fast);
        PR_HIP(hipMemcpyAsync(a.data(), sde->a, sizeof(double) * sde->d_fast, hipMemcpyDeviceToHost, st));
        PR_HIP(hipStreamSynchronize(st));
        double s = 0.0;
        for (double v : a) s += v;
        abar = s / sde->d_fast;
    }
    const double k2 = sde->c1 + sde->lambda * (1.0 - abar);
    const double beta = sde->beta, dbar = 1.0 / beta;
    auto V = [&](double x) { return sde->c3 * x * x * x * x / 4.0 + k2 * x * x / 2.0; };
    std::vector<double> g(I), a(I + 1, 0.0);
    for (int i = 0; i < I; ++i) {
        const double m = grid->x_lo + (i + 0.5) * h;
        g[i] = h * std::exp(-beta * V(m));
    }
    for (int i = 1; i < I; ++i) {
        const double e = grid->x_lo + i * h;
        a[i] = dbar * std::exp(-beta * V(e)) / h;
    }
    lo.assign(I, 0.0);
    di.assign(I, 0.0);
    up.assign(I, 0.0);
    for (int i = 0; i < I; ++i) {
        di[i] = -(a[i] + a[i + 1]) / g[i];
        if (i + 1 < I) up[i] = a[i + 1] / g[i + 1];
        if (i >= 1) lo[i] = a[i] / g[i - 1];
    }
    return PR_OK;
}

int coarse_create(const pr_sde *sde, const pr_schedule *sch, const pr_grid *grid, hipStream_t st,
                  Coarse **out) {
    std::vector<double> lo, di, up;
    PR_CHECK(make_generator(sde, grid, lo, di, up, st));
    return coarse_create_tridiag(lo, di, up, sch, grid, st, out);
}

int coarse_create_tridiag(const std::vector<double> &lo, const std::vector<double> &di,
                          const std::vector<double> &up, const pr_schedule *sch, const pr_grid *grid, hipStream_t st,
                          Coarse **out) {
    const int I = grid->n_cells;
    const double h = (grid->x_hi - grid->x_lo) / I;
    Coarse *c = new Coarse();
    c->g = GridDev{I, grid->n_q, grid->x_lo, h};
    c->n_slices = sch->n_slices;
    std::vector<int> ids(sch->n_slices);
    std::vector<int64_t> lens;
    for (int n = 0; n < sch->n_slices; ++n) {
        const int64_t L = slice_begin(sch->total_steps, sch->n_slices, n + 1) -
                          slice_begin(sch->total_steps, sch->n_slices, n);
        int id = -1;
        for (size_t t = 0; t < lens.size(); ++t)
            if (lens[t] == L) id = (int)t;
        if (id < 0) {
            id = (int)lens.size();
            lens.push_back(L);
            c->taus.push_back((double)L * sch->dt);
        }
        ids[n] = id;
    }
    c->n_tau = (int)lens.size();
    const int64_t nn = (int64_t)I * I;
    auto fail = [&](int code) {
        if (c->E) (void)hipFree(c->E);
        if (c->tau_id) (void)hipFree(c->tau_id);
        if (c->rho_a) (void)hipFree(c->rho_a);
        delete c;
        return code;
    };
    if (hipMalloc(&c->E, sizeof(double) * nn * c->n_tau) != hipSuccess ||
        hipMalloc(&c->tau_id, sizeof(int) * sch->n_slices) != hipSuccess ||
        hipMalloc(&c->rho_a, sizeof(double) * (size_t)I * sch->n_slices * 2) != hipSuccess) {
        set_error("device allocation of the coarse propagator failed");
        return fail(PR_E_NOMEM);
    }
    c->rho_b = c->rho_a + (size_t)I * sch->n_slices;
    if (hipMemcpyAsync(c->tau_id, ids.data(), sizeof(int) * sch->n_slices, hipMemcpyHostToDevice, st) != hipSuccess) {
        set_error("copy of the slice table failed");
        return fail(PR_E_HIP);
    }
    double *w = nullptr;
    if (hipMalloc(&w, sizeof(double) * nn * 3) != hipSuccess) {
        set_error("device allocation of the exponential workspace failed");
        return fail(PR_E_NOMEM);
    }
    for (int t = 0; t < c->n_tau; ++t) {
        const int s = build_expm(lo, di, up, I, c->taus[t], c->E + nn * t, w, w + nn, w + 2 * nn, st);
        if (s != PR_OK) {
            (void)hipFree(w);
            return fail(s);
        }
    }
    (void)hipFree(w);
    (void)hipGetDevice(&c->device);
    *out = c;
    return PR_OK;
}

static size_t lds_knots_to_masses(const GridDev &g) { return sizeof(double) * (g.nq + 1 + g.cells + 1); }
static size_t lds_masses_to_knots(const GridDev &g) { return sizeof(double) * (2 * g.cells + 1); }
static size_t lds_qf_jump(const GridDev &g) {
    return sizeof(double) * (2 * g.cells + 1 + 2 * (g.nq + 1)) + 2 * sizeof(int) * (g.nq + 1);
}

// Batched coarse step of slices [first, first+count): q_in -> q_out.
int coarse_step(const Coarse *c, int first, int count, const double *q_in, int in_stride, double *q_out,
                int out_stride, double *rho_out, hipStream_t st) {
    if (count == 0) return PR_OK;
    const GridDev &g = c->g;
    double *ra = c->rho_a, *rb = rho_out ? rho_out : c->rho_b;
    hipLaunchKernelGGL(knots_to_masses, dim3(count), dim3(256), lds_knots_to_masses(g), st, q_in, in_stride, ra, g);
    PR_LAUNCHED();
    hipLaunchKernelGGL(apply_expm, dim3((g.cells + 3) / 4, count), dim3(256), sizeof(double) * g.cells, st,
                       (const double *)c->E, (const int *)c->tau_id, first, (const double *)ra, rb, g.cells);
    PR_LAUNCHED();
    hipLaunchKernelGGL(masses_to_knots, dim3(count), dim3(256), lds_masses_to_knots(g), st, (const double *)rb,
                       q_out, out_stride, g);
    PR_LAUNCHED();
    return PR_OK;
}

// One link of the serial chain: q_next = J(C_n(q_cur), q_f, q_cs).
int coarse_jump(const Coarse *c, int n, const double *q_cur, const double *qf, const double *qcs, double *q_next,
                double *qc_out, hipStream_t st) {
    const GridDev &g = c->g;
    hipLaunchKernelGGL(apply_expm_knots, dim3((g.cells + 3) / 4), dim3(256),
                       sizeof(double) * (g.nq + 1 + 2 * g.cells + 1), st, (const double *)c->E,
                       (const int *)c->tau_id, n, q_cur, c->rho_b, g);
    PR_LAUNCHED();
    hipLaunchKernelGGL(qf_and_jump, dim3(1), dim3(256), lds_qf_jump(g), st, (const double *)c->rho_b, qf, qcs, q_next,
                       qc_out, g);
    PR_LAUNCHED();
    return PR_OK;
}

// rho_out[s] = max(E_{first+s} rho_in[s], 0) for s < count (cell masses).
int coarse_apply(const Coarse *c, int first, int count, const double *rho_in, double *rho_out, hipStream_t st) {
    if (count == 0) return PR_OK;
    const GridDev &g = c->g;
    hipLaunchKernelGGL(apply_expm, dim3((g.cells + 3) / 4, count), dim3(256), sizeof(double) * g.cells, st,
                       (const double *)c->E, (const int *)c->tau_id, first, rho_in, rho_out, g.cells);
    PR_LAUNCHED();
    return PR_OK;
}

int coarse_grid_nq(const Coarse *c) { return c->g.nq; }
int coarse_n_slices(const Coarse *c) { return c->n_slices; }
int coarse_grid_cells(const Coarse *c) { return c->g.cells; }

void coarse_free(Coarse *c) {
    if (!c) return;
    (void)hipFree(c->E);
    (void)hipFree(c->tau_id);
    (void)hipFree(c->rho_a);
    delete c;
}

}  // namespace pr

using namespace pr;

extern "C" int pr_coarse_create(const pr_sde *sde, const pr_schedule *sched, const pr_grid *grid, void *stream,
                                void **coarse) {
    clear_error();
    PR_CHECK(check_sde(sde));
    PR_CHECK(check_schedule(sched));
    PR_CHECK(check_grid(grid));
    PR_REQUIRE(coarse != nullptr, "coarse is NULL");
    Coarse *c = nullptr;
    PR_CHECK(coarse_create(sde, sched, grid, as_stream(stream), &c));
    *coarse = c;
    return PR_OK;
}

extern "C" int pr_coarse_fp_step(const void *coarse, int slice_first, int slice_count, const double *q_in,
                                 double *q_out, double *rho_out, void *stream) {
    clear_error();
    PR_REQUIRE(coarse != nullptr, "coarse is NULL");
    const Coarse *c = (const Coarse *)coarse;
    PR_REQUIRE(slice_first >= 0 && slice_count >= 0 && slice_first + slice_count <= c->n_slices,
               "slices outside the schedule");
    PR_REQUIRE(slice_count <= 65535, "at most 65535 slices per call");
    PR_REQUIRE(slice_count == 0 || (q_in && q_out), "q_in and q_out must be non-NULL");
    return coarse_step(c, slice_first, slice_count, q_in, c->g.nq + 1, q_out, c->g.nq + 1, rho_out,
                       as_stream(stream));
}

extern "C" int pr_coarse_matrix(const void *coarse, int slice, const double **E) {
    clear_error();
    PR_REQUIRE(coarse != nullptr && E != nullptr, "coarse and E must be non-NULL");
    const Coarse *c = (const Coarse *)coarse;
    PR_REQUIRE(slice >= 0 && slice < c->n_slices, "slice out of range");
    int id = 0;
    PR_HIP(hipMemcpy(&id, c->tau_id + slice, sizeof(int), hipMemcpyDeviceToHost));
    *E = c->E + (int64_t)id * c->g.cells * c->g.cells;
    return PR_OK;
}

extern "C" int pr_coarse_destroy(void *coarse) {
    clear_error();
    coarse_free((Coarse *)coarse);
    return PR_OK;
}

extern "C" int pr_quantile_jump(const double *q_c_next, const double *q_f, const double *q_c_star, int k, int n_q,
                                double *q_out, void *stream) {
    clear_error();
    PR_REQUIRE(k >= 0, "k must be >= 0");
    PR_REQUIRE(n_q >= 1 && n_q <= 2047, "n_q must be in [1, 2047]");
    if (k == 0) return PR_OK;
    PR_REQUIRE(q_c_next && q_f && q_c_star && q_out, "the knot arrays must be non-NULL");
    const int L = n_q + 1;
    hipLaunchKernelGGL(quantile_jump_rows, dim3((unsigned)k), dim3(256), (sizeof(double) * 2 + sizeof(int) * 2) * L,
                       as_stream(stream), q_c_next, q_f, q_c_star, q_out, L);
    PR_LAUNCHED();
    return PR_OK;
}
