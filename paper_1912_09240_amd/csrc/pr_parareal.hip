// Micro-macro parareal driver (Sec. 3.2.3-3.2.4) with the quantile iterator
// (Sec. 4.4) and fast-marginal matching (Sec. 5.1).
//
// State: two ensemble buffers (ping-pong), each holding the N+1 time points
// x[t][P], y[t][d][P], t = 0..N; t = 0 is the initial ensemble in both.  An
// iteration k -> k+1 reads the states X_k^n of one buffer and writes
// X_{k+1}^{n+1} into the other:
//   1. fine propagation of all slices at once (slice n: X_k^n -> Xbar^{n+1});
//   2. restriction of every Xbar^{n+1} (knots q_f, ranks for matching);
//   3. coarse propagation of every slice from R(X_k^n) (or from q_k^n when
//      the coarse results are reused) in parallel -> q_c^*;
//   4. the serial chain q_{k+1}^{n+1} = J(C_n(q_{k+1}^n), q_f^{n+1}, q_c^{*,n+1});
//   5. matching of every Xbar^{n+1} to q_{k+1}^{n+1} (in place);
//   6. knots of the new states (next coarse input and the error to a
//      reference).
#include <vector>

#include "pr_internal.hpp"

namespace pr {

struct Parareal {
    pr_sde sde;
    pr_schedule sch;
    pr_grid grid;
    uint64_t seed;
    uint32_t inst;
    int64_t n;
    int flags;
    int K, Q, D, esz;
    Coarse *coarse = nullptr;
    double *a = nullptr;             // owned copy of the coupling coefficients
    char *x[2] = {nullptr, nullptr};  // [K+1][n]
    char *y[2] = {nullptr, nullptr};  // [K+1][D][n]
    double *q = nullptr;     // [K+1][Q+1]  coarse-level states q_k^n
    double *qn = nullptr;    // [K+1][Q+1]  next coarse-level states
    double *qR = nullptr;    // [K+1][Q+1]  knots of the current states
    double *qf = nullptr;    // [K+1][Q+1]  knots of the fine results (index n+1)
    double *qcs = nullptr;   // [K+1][Q+1]  coarse results of the previous states
    uint32_t *rank = nullptr;  // [K][n] ranks of the fine results / of X0
    double *err = nullptr;   // [2]
    int *flag = nullptr;     // set where the knots of the new states need a sort
    int *flag_host = nullptr;  // pinned copy of it
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int cur = 0;
    int k = 0;
    int knot_sorts = 0;  // iterations whose new knots needed the sort
    hipEvent_t ev[PR_PH_COUNT + 1] = {};
    double ph_ms[PR_PH_COUNT] = {};
    int timed = 0;

    char *xs(int b, int t) const { return x[b] + (size_t)t * n * esz; }
    char *ys(int b, int t) const { return y[b] + (size_t)t * D * n * esz; }
    double *qrow(double *base, int t) const { return base + (size_t)t * (Q + 1); }
};

static void parareal_free(Parareal *h) {
    if (!h) return;
    if (h->coarse) coarse_free(h->coarse);
    void *ptrs[] = {h->a, h->x[0], h->x[1], h->y[0], h->y[1], h->q, h->qn, h->qR, h->qf, h->qcs,
                    h->rank, h->err, h->ws};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (h->flag) (void)hipFree(h->flag);
    if (h->flag_host) (void)hipHostFree(h->flag_host);
    for (hipEvent_t e : h->ev)
        if (e) (void)hipEventDestroy(e);
    delete h;
}

__global__ void knot_error(const double *__restrict__ qR, const double *__restrict__ qref, int K, int nq,
                           double *__restrict__ err) {
    __shared__ double e[1024];
    for (int t = threadIdx.x; t <= K; t += blockDim.x) {
        double s = 0.0;
        for (int j = 0; j <= nq; ++j) {
            const double d = qR[(size_t)t * (nq + 1) + j] - qref[(size_t)t * (nq + 1) + j];
            s += d * d;
        }
        e[t] = sqrt(s / (double)(nq + 1));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int t = 0; t <= K; ++t) m = e[t] > m ? e[t] : m;
        err[0] = e[K];
        err[1] = m;
    }
}

#define PR_ALLOC(ptr, bytes)                                                  \
    do {                                                                      \
        if (hipMalloc((void **)&(ptr), (bytes)) != hipSuccess) {              \
            set_error("device allocation of %zu bytes failed", (size_t)(bytes)); \
            parareal_free(h);                                                 \
            return PR_E_NOMEM;                                                \
        }                                                                     \
    } while (0)

#define PR_TRY(expr)                 \
    do {                             \
        int s_ = (expr);             \
        if (s_ != PR_OK) {           \
            parareal_free(h);        \
            return s_;               \
        }                            \
    } while (0)

// Knots of the states at t = first .. first+count-1 of buffer b into qR.
static int restrict_states(Parareal *h, int b, int first, int count, hipStream_t st) {
    return restrict_quantiles(h->xs(b, first), h->sde.precision, h->n, count, h->Q, nullptr,
                              h->qrow(h->qR, first), nullptr, nullptr, nullptr, nullptr, nullptr, h->ws, st);
}

int parareal_create(const pr_sde *sde_in, const pr_schedule *sch, const pr_grid *grid, uint64_t seed,
                    uint32_t inst, int64_t n, int flags, hipStream_t st, Parareal **out) {
    Parareal *h = new Parareal();
    h->sde = *sde_in;
    h->sch = *sch;
    h->grid = *grid;
    h->seed = seed;
    h->inst = inst;
    h->n = n;
    h->flags = flags;
    h->K = sch->n_slices;
    h->Q = grid->n_q;
    h->D = sde_in->d_fast;
    h->esz = sde_in->precision == PR_F64 ? 8 : 4;
    const int K = h->K, Q = h->Q, D = h->D;
    if (sde_in->a) {
        PR_ALLOC(h->a, sizeof(double) * D);
        PR_TRY(hipMemcpyAsync(h->a, sde_in->a, sizeof(double) * D, hipMemcpyDeviceToDevice, st) == hipSuccess
                   ? PR_OK
                   : PR_E_HIP);
        h->sde.a = h->a;
    }
    const size_t xb = (size_t)(K + 1) * n * h->esz, yb = xb * D, qb = sizeof(double) * (K + 1) * (Q + 1);
    for (int b = 0; b < 2; ++b) {
        PR_ALLOC(h->x[b], xb);
        PR_ALLOC(h->y[b], yb);
    }
    PR_ALLOC(h->q, qb);
    PR_ALLOC(h->qn, qb);
    PR_ALLOC(h->qR, qb);
    PR_ALLOC(h->qf, qb);
    PR_ALLOC(h->qcs, qb);
    PR_ALLOC(h->rank, sizeof(uint32_t) * (size_t)K * n);
    PR_ALLOC(h->err, sizeof(double) * 2);
    PR_ALLOC(h->flag, sizeof(int));
    PR_TRY(hipHostMalloc((void **)&h->flag_host, sizeof(int), hipHostMallocDefault) == hipSuccess ? PR_OK
                                                                                                   : PR_E_NOMEM);
    h->ws_bytes = restrict_ws(n, K + 1, h->sde.precision);
    PR_ALLOC(h->ws, h->ws_bytes);
    PR_TRY(coarse_create(&h->sde, sch, grid, st, &h->coarse));
    if (flags & PR_PROFILE)
        for (hipEvent_t &e : h->ev)
            PR_TRY(hipEventCreate(&e) == hipSuccess ? PR_OK : PR_E_HIP);

    // initial ensemble in slot 0 of both buffers
    PR_TRY(init_ensemble(&h->sde, seed, inst, n, h->xs(0, 0), h->ys(0, 0), st));
    PR_TRY(hipMemcpyAsync(h->xs(1, 0), h->xs(0, 0), (size_t)n * h->esz, hipMemcpyDeviceToDevice, st) == hipSuccess
               ? PR_OK : PR_E_HIP);
    PR_TRY(hipMemcpyAsync(h->ys(1, 0), h->ys(0, 0), (size_t)D * n * h->esz, hipMemcpyDeviceToDevice, st) == hipSuccess
               ? PR_OK : PR_E_HIP);
    // zeroth iteration: q_0^0 = R(X0) (with X0's ranks), q_0^{n+1} = C_n(q_0^n)
    PR_TRY(restrict_quantiles(h->xs(0, 0), h->sde.precision, n, 1, Q, nullptr, h->q, h->rank, nullptr, nullptr,
                              nullptr, nullptr, h->ws, st));
    for (int s = 0; s < K; ++s)
        PR_TRY(coarse_step(h->coarse, s, 1, h->qrow(h->q, s), Q + 1, h->qrow(h->q, s + 1), Q + 1, nullptr, st));
    // X_0^n = M(q_0^n; X0) for n = 1..K; fast variables copied from X0
    MatchArgs ma{h->qrow(h->q, 1), Q + 1, h->q, 0, h->rank, 0, h->xs(0, 0), 0, h->xs(0, 1), n};
    PR_TRY(match_strided(ma, n, K, Q, h->sde.precision, st));
    for (int t = 1; t <= K; ++t)
        PR_TRY(hipMemcpyAsync(h->ys(0, t), h->ys(0, 0), (size_t)D * n * h->esz, hipMemcpyDeviceToDevice, st) ==
                       hipSuccess ? PR_OK : PR_E_HIP);
    PR_TRY(restrict_states(h, 0, 0, K + 1, st));
    if (hipStreamSynchronize(st) != hipSuccess) {
        set_error("zeroth iteration failed on the device");
        parareal_free(h);
        return PR_E_HIP;
    }
    *out = h;
    return PR_OK;
}

int parareal_iterate(Parareal *h, int n_iter, const double *q_ref, double *err_out, hipStream_t st) {
    const int K = h->K, Q = h->Q;
    const int64_t n = h->n;
    const bool prof = (h->flags & PR_PROFILE) != 0;
    auto mark = [&](int i) -> int {
        if (prof) PR_HIP(hipEventRecord(h->ev[i], st));
        return PR_OK;
    };
    for (int it = 0; it < n_iter; ++it) {
        const int c = h->cur, nx = 1 - c;
        PR_CHECK(mark(0));
        // 1. fine: slice s reads X_k^s from buffer c, writes Xbar^{s+1} into buffer nx
        int first = 0;
        if (h->flags & PR_SKIP_CONVERGED) {
            first = h->k < K ? h->k : K;  // states at t <= k are exact: copy them
            if (first > 0) {
                PR_HIP(hipMemcpyAsync(h->xs(nx, 1), h->xs(c, 1), (size_t)first * n * h->esz, hipMemcpyDeviceToDevice, st));
                PR_HIP(hipMemcpyAsync(h->ys(nx, 1), h->ys(c, 1), (size_t)first * h->D * n * h->esz,
                                      hipMemcpyDeviceToDevice, st));
            }
        }
        PR_CHECK(fine_propagate(&h->sde, &h->sch, h->seed, h->inst, n, first, K - first, h->xs(c, first),
                                h->ys(c, first), h->xs(nx, first + 1), h->ys(nx, first + 1), st));
        PR_CHECK(mark(1));
        // 2. restriction of the fine results: q_f^{s+1}, ranks
        PR_CHECK(restrict_quantiles(h->xs(nx, 1), h->sde.precision, n, K, Q, nullptr, h->qrow(h->qf, 1), h->rank,
                                    nullptr, nullptr, nullptr, nullptr, h->ws, st));
        PR_CHECK(mark(2));
        // 3. coarse propagation of every slice from the previous states
        const double *cin = (h->flags & PR_REUSE_COARSE) ? h->q : h->qR;
        PR_CHECK(coarse_step(h->coarse, 0, K, cin, Q + 1, h->qrow(h->qcs, 1), Q + 1, nullptr, st));
        PR_CHECK(mark(3));
        // 4. serial chain
        PR_HIP(hipMemcpyAsync(h->qn, h->q, sizeof(double) * (Q + 1), hipMemcpyDeviceToDevice, st));
        for (int s = 0; s < K; ++s)
            PR_CHECK(coarse_jump(h->coarse, s, h->qrow(h->qn, s), h->qrow(h->qf, s + 1), h->qrow(h->qcs, s + 1),
                                 h->qrow(h->qn, s + 1), nullptr, st));
        PR_CHECK(mark(4));
        // 5. matching of the fine results, in place
        MatchArgs ma{h->qrow(h->qn, 1), Q + 1, h->qrow(h->qf, 1), Q + 1, h->rank, n, h->xs(nx, 1), n,
                     h->xs(nx, 1), n};
        PR_CHECK(match_strided(ma, n, K, Q, h->sde.precision, st));
        PR_CHECK(mark(5));
        std::swap(h->q, h->qn);
        // 6. knots of the new states: order statistics of the matched values
        // found from the fine results' sort (which the restriction left in
        // the workspace), or a sort of the new states where that fails
        const int mk = matched_knots(h->ws, h->sde.precision, n, K, Q, h->qrow(h->q, 1), Q + 1, h->qrow(h->qf, 1),
                                     Q + 1, h->qrow(h->qR, 1), h->flag, st);
        if (mk != PR_OK && mk != PR_E_UNSUPPORTED) return mk;
        bool sort_new = mk == PR_E_UNSUPPORTED;
        if (!sort_new) {
            PR_HIP(hipMemcpyAsync(h->flag_host, h->flag, sizeof(int), hipMemcpyDeviceToHost, st));
            PR_HIP(hipStreamSynchronize(st));
            sort_new = *h->flag_host != 0;
        }
        if (sort_new) {
            PR_CHECK(restrict_states(h, nx, 1, K, st));
            ++h->knot_sorts;
        }
        h->cur = nx;
        h->k += 1;
        if (q_ref) {
            hipLaunchKernelGGL(knot_error, dim3(1), dim3(256), 0, st, (const double *)h->qR, q_ref, K, Q, h->err);
            PR_LAUNCHED();
        }
        PR_CHECK(mark(6));
        if (q_ref && err_out) {
            PR_HIP(hipMemcpyAsync(err_out + 2 * it, h->err, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
            PR_HIP(hipStreamSynchronize(st));
        }
        if (prof) {
            PR_HIP(hipEventSynchronize(h->ev[PR_PH_COUNT]));
            for (int p = 0; p < PR_PH_COUNT; ++p) {
                float ms = 0.f;
                PR_HIP(hipEventElapsedTime(&ms, h->ev[p], h->ev[p + 1]));
                h->ph_ms[p] += ms;
            }
            h->timed += 1;
        }
    }
    return PR_OK;
}

}  // namespace pr

using namespace pr;

extern "C" int pr_parareal_create(const pr_sde *sde, const pr_schedule *sched, const pr_grid *grid, uint64_t seed,
                                  uint32_t instance, int64_t n, int flags, void *stream, void **h) {
    clear_error();
    PR_CHECK(check_sde(sde));
    PR_CHECK(check_schedule(sched));
    PR_CHECK(check_grid(grid));
    PR_REQUIRE(h != nullptr, "h is NULL");
    PR_REQUIRE(n >= 1 && n <= 0xFFFFFFFFll, "n must be in [1, 2^32)");
    PR_REQUIRE(sched->n_slices <= 1023, "at most 1023 slices");
    PR_REQUIRE((flags & ~(PR_REUSE_COARSE | PR_SKIP_CONVERGED | PR_PROFILE)) == 0, "unknown flags");
    Parareal *p = nullptr;
    PR_CHECK(parareal_create(sde, sched, grid, seed, instance, n, flags, as_stream(stream), &p));
    *h = p;
    return PR_OK;
}

extern "C" int pr_parareal_iterate(void *h, int n_iter, const double *q_ref, double *err_out, void *stream) {
    clear_error();
    PR_REQUIRE(h != nullptr, "h is NULL");
    PR_REQUIRE(n_iter >= 0, "n_iter must be >= 0");
    PR_REQUIRE(err_out == nullptr || q_ref != nullptr, "err_out needs q_ref");
    return parareal_iterate((Parareal *)h, n_iter, q_ref, err_out, as_stream(stream));
}

extern "C" int pr_parareal_state(void *hv, int t, void *x, void *y, double *q, void *stream) {
    clear_error();
    PR_REQUIRE(hv != nullptr, "h is NULL");
    Parareal *h = (Parareal *)hv;
    PR_REQUIRE(t >= 0 && t <= h->K, "t must be in [0, %d]", h->K);
    hipStream_t st = as_stream(stream);
    if (x) PR_HIP(hipMemcpyAsync(x, h->xs(h->cur, t), (size_t)h->n * h->esz, hipMemcpyDeviceToDevice, st));
    if (y) PR_HIP(hipMemcpyAsync(y, h->ys(h->cur, t), (size_t)h->D * h->n * h->esz, hipMemcpyDeviceToDevice, st));
    if (q) PR_HIP(hipMemcpyAsync(q, h->qrow(h->qR, t), sizeof(double) * (h->Q + 1), hipMemcpyDeviceToDevice, st));
    return PR_OK;
}

extern "C" int pr_parareal_iteration(const void *h) { return h ? ((const Parareal *)h)->k : -1; }

extern "C" int pr_parareal_knot_sorts(const void *h) { return h ? ((const Parareal *)h)->knot_sorts : -1; }

extern "C" int pr_parareal_profile(const void *hv, double *ms_out, int *iterations) {
    clear_error();
    PR_REQUIRE(hv != nullptr && ms_out != nullptr, "h and ms_out must be non-NULL");
    const Parareal *h = (const Parareal *)hv;
    PR_REQUIRE(h->flags & PR_PROFILE, "handle was created without PR_PROFILE");
    for (int p = 0; p < PR_PH_COUNT; ++p) ms_out[p] = h->ph_ms[p];
    if (iterations) *iterations = h->timed;
    return PR_OK;
}

extern "C" int pr_parareal_destroy(void *h) {
    clear_error();
    parareal_free((Parareal *)h);
    return PR_OK;
}
