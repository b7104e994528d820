// Matching that preserves the fast marginal (Sec. 5.1, eq. (transformation)),
// written as a perturbation of the prior: the prior's own mid-rank cdf value
// u = (rank + 1/2)/P is pushed through q_target and pulled back through
// q_prior, both piecewise linear on the knots p_j = j/Q, so
//   X = Xbar + (1-w) d_j + w d_{j+1},  d = q_target - q_prior.
// Streaming kernel: reads Xbar and rank in particle order, writes X in
// particle order (20 bytes per particle in FP64); the knot differences of the
// segment sit in LDS.
#include "pr_internal.hpp"

namespace pr {

constexpr int MT_THREADS = 256;
constexpr int MT_PPT = 4;  // particles per thread

template <typename T>
__global__ void __launch_bounds__(MT_THREADS) match_kernel(MatchArgs a, int64_t n, int nq) {
#pragma clang fp contract(off)
    extern __shared__ double dk[];
    const int seg = blockIdx.y;
    for (int j = threadIdx.x; j <= nq; j += MT_THREADS)
        dk[j] = a.qt[seg * a.qt_stride + j] - a.qp[seg * a.qp_stride + j];
    __syncthreads();
    const double nd = (double)n;
    const double Q = (double)nq;
    const uint32_t *rank = a.rank + seg * a.rank_stride;
    const T *xin = (const T *)a.xin + seg * a.xin_stride;
    T *xout = (T *)a.xout + seg * a.xout_stride;
    const int64_t p0 = (int64_t)blockIdx.x * MT_THREADS * MT_PPT + threadIdx.x;
#pragma unroll
    for (int q = 0; q < MT_PPT; ++q) {
        const int64_t p = p0 + (int64_t)q * MT_THREADS;
        if (p >= n) break;
        xout[p] = matched_value<T>(xin[p], rank[p], dk, nd, Q);
    }
}

int match_strided(const MatchArgs &a, int64_t n, int k, int nq, int precision, hipStream_t st) {
    if (n == 0 || k == 0) return PR_OK;
    const int64_t per_block = (int64_t)MT_THREADS * MT_PPT;
    const dim3 grid((unsigned)((n + per_block - 1) / per_block), (unsigned)k);
    const size_t lds = (size_t)(nq + 1) * sizeof(double);
    if (precision == PR_F64)
        hipLaunchKernelGGL(match_kernel<double>, grid, dim3(MT_THREADS), lds, st, a, n, nq);
    else
        hipLaunchKernelGGL(match_kernel<float>, grid, dim3(MT_THREADS), lds, st, a, n, nq);
    PR_LAUNCHED();
    return PR_OK;
}

int match_quantiles(const double *qt, const double *qp, const uint32_t *rank, int64_t n, int k, int nq,
                    const void *xin, void *xout, int precision, hipStream_t st) {
    const int64_t qs = nq + 1;
    MatchArgs a{qt, qs, qp, qs, rank, n, xin, n, xout, n};
    return match_strided(a, n, k, nq, precision, st);
}

}  // namespace pr

using namespace pr;

extern "C" int pr_match_quantiles(const double *q_target, const double *q_prior, const uint32_t *rank,
                                  int64_t n, int k, int n_q, const void *x_prior, void *x_out, int precision,
                                  void *stream) {
    clear_error();
    PR_REQUIRE(valid_precision(precision), "precision must be 64 or 32");
    PR_REQUIRE(n >= 0 && n <= 0xFFFFFFFFll, "n must be in [0, 2^32)");
    PR_REQUIRE(k >= 0 && k <= 65535, "k must be in [0, 65535]");
    PR_REQUIRE(n_q >= 1 && n_q <= 8191, "n_q must be in [1, 8191]");
    PR_REQUIRE(n == 0 || k == 0 ||
                   (q_target && q_prior && rank && x_prior && x_out),
               "pointers must be non-NULL");
    return match_quantiles(q_target, q_prior, rank, n, k, n_q, x_prior, x_out, precision, as_stream(stream));
}
