// Histogram-state micro-macro parareal: the macroscopic state is the vector
// of cell masses of the slow variable (eq. (integral), eq. (binning)).
//
//   restriction  weighted histograms of many ensembles.  With equal weights
//                w0 = RN(1/P) a cell holds RN(count w0); with weights, every
//                weight is turned into a 128-bit fixed-point number with
//                2^-112 units (exact for weights in [2^-60, 2^15)), the sums
//                are exact integers and the mass is the sum rounded once.
//   iterators    additive, multiplicative, rotation (Sec. 4.1-4.3) and the
//                quantile iterator on the union of the three cdfs' edge levels
//                (Sec. 4.4), each on one slice per workgroup; every sum over
//                the cells runs left to right.
//   matchings    fast-marginal matching on piecewise-linear cdfs
//                (eq. (transformation)); conditional matching by reweighting,
//                optionally followed by stratified resampling (Sec. 5.2) with
//                cumulative weights in 64-bit fixed point, so that every slot
//                decision is an exact integer comparison.
//   driver       zeroth and generic iterations (Sec. 3.2.3-3.2.4) with the
//                fine propagator, the coarse exponentials and the serial
//                chain of coarse step + iterator.
//
// Conventions shared with the rest of the library: cell i of the grid is
// [x_i, x_{i+1}) with index floor((x - x_lo) I / (x_hi - x_lo)) clamped to
// the grid, x_i = x_lo + i h; a histogram's cdf at the edges is the
// left-to-right running sum of its masses; the quantile of a histogram at a
// level is the midpoint of the set where the piecewise-linear cdf takes that
// level, the right end of it at level 0 and the left end at the total mass.
#include <algorithm>
#include <vector>

#include "pr_chem.hpp"
#include "pr_coarse_dev.hpp"
#include "pr_internal.hpp"

namespace pr {

typedef unsigned __int128 u128;

constexpr int HB_THREADS = 256;
constexpr int HB_ITEMS = 8;
constexpr int HB_TILE = HB_THREADS * HB_ITEMS;  // particles per tile of the resampling
constexpr int HB_MAX_CELLS = 1024;
constexpr int JQ_THREADS = 1024;  // the quantile iterator: one workgroup per slice along a serial chain
constexpr int FIX_W = 112;  // fraction bits of the histogram weights
constexpr uint32_t TAG_RESAMPLE = 4u;

// ---------------------------------------------------------------------------
// Fixed point.
// ---------------------------------------------------------------------------
// floor(w 2^scale) for w >= 0 (w < 2^(127 - scale)); 0 for w <= 0.
__host__ __device__ inline u128 fix_floor(double w, int scale) {
    const uint64_t b = __builtin_bit_cast(uint64_t, w);
    if (b >> 63) return 0;
    const int E = (int)((b >> 52) & 0x7FF);
    if (E == 0) return 0;  // zero, or below 2^-1022: far below one unit
    const uint64_t m = (b & ((1ull << 52) - 1)) | (1ull << 52);
    const int s = E - 1075 + scale;  // w 2^scale = m 2^s
    if (s >= 0) return (u128)m << s;
    if (s <= -64) return 0;
    return (u128)(m >> (-s));
}

__host__ __device__ inline int clz128(u128 v) {
    const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    return hi ? __builtin_clzll(hi) : 64 + __builtin_clzll(lo);
}

// v 2^-scale rounded to the nearest double (ties to even).
__host__ __device__ inline double fix_to_double(u128 v, int scale) {
    if (v == 0) return 0.0;
    const int msb = 127 - clz128(v);
    if (msb <= 52) return __builtin_ldexp((double)(uint64_t)v, -scale);
    int sh = msb - 52;
    uint64_t mant = (uint64_t)(v >> sh);
    const u128 rem = v & ((((u128)1) << sh) - 1);
    const u128 half = ((u128)1) << (sh - 1);
    if (rem > half || (rem == half && (mant & 1ull))) {
        mant += 1;
        if (mant == (1ull << 53)) {
            mant >>= 1;
            sh += 1;
        }
    }
    return __builtin_ldexp((double)mant, sh - scale);
}

// floor(v / d), d < 2^32.
__host__ __device__ inline u128 udiv128_32(u128 v, uint32_t d) {
    const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    const uint64_t qh = hi / d, r = hi % d;
    const uint64_t t1 = (r << 32) | (lo >> 32);
    const uint64_t q1 = t1 / d, r1 = t1 % d;
    const uint64_t t0 = (r1 << 32) | (lo & 0xFFFFFFFFull);
    const uint64_t q0 = t0 / d;
    return ((u128)qh << 64) | ((u128)q1 << 32) | (u128)q0;
}

// Resampling weight: floor(W 2^64), capped at 2^64 - 1.
__host__ __device__ inline uint64_t fix_weight(double w) {
    if (!(w < 1.0)) return w >= 1.0 ? ~0ull : 0ull;
    return (uint64_t)fix_floor(w, 64);
}

// U_j = floor(j T / P) + floor(k_j T / (P 2^32)), with T = qT P + rT:
//   floor(j T / P)          = j qT + floor(j rT / P)
//   floor(k T / (P 2^32))   = (k qT + floor(k rT / P)) >> 32
// (j rT and k rT stay below 2^64 with quotients below 2^32).
struct SlotConst {
    u128 qT;
    uint64_t rT;
    double inv_p;  // 1/P, rounded
};

// floor(a / P) for a < 2^64 whose quotient is below 2^32: the double
// estimate a (1/P) is within a few units, the remainder fixes it exactly.
__host__ __device__ inline uint64_t floor_div_p(uint64_t a, uint32_t P, double inv_p) {
    uint64_t q = (uint64_t)((double)a * inv_p);
    int64_t r = (int64_t)(a - q * (uint64_t)P);
    while (r < 0) {
        --q;
        r += (int64_t)P;
    }
    while (r >= (int64_t)P) {
        ++q;
        r -= (int64_t)P;
    }
    return q;
}

__host__ __device__ inline u128 slot_level(uint64_t j, uint32_t kj, const SlotConst &c, uint32_t P) {
    const u128 a = (u128)j * c.qT + (u128)floor_div_p(j * c.rT, P, c.inv_p);
    const u128 b = ((u128)kj * c.qT + (u128)floor_div_p((uint64_t)kj * c.rT, P, c.inv_p)) >> 32;
    return a + b;
}

__device__ inline uint32_t slot_draw(Key key, uint32_t inst, uint32_t j, uint32_t t, int det) {
    if (det) return 0x80000000u;
    return noise_block(key, inst, TAG_RESAMPLE, 0u, j, t).w0;
}

// ---------------------------------------------------------------------------
// Grid helpers.
// ---------------------------------------------------------------------------
struct HGrid {
    int cells;
    double lo, h, inv_h;
};

__device__ __forceinline__ double hedge(const HGrid &g, int i) {
#pragma clang fp contract(off)
    return g.lo + (double)i * g.h;
}

__device__ __forceinline__ int hcell(const HGrid &g, double x) {
#pragma clang fp contract(off)
    double c = floor((x - g.lo) * g.inv_h);
    c = fmin(fmax(c, 0.0), (double)(g.cells - 1));
    return (int)c;
}

// first index in [0, n) with a[i] >= v (n if none)
__device__ __forceinline__ int lower_bound_d(const double *a, int n, double v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// first index in [0, n) with a[i] > v (n if none)
__device__ __forceinline__ int upper_bound_d(const double *a, int n, double v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Quantile of the histogram rho (cdf c at the I + 1 edges) at a level p in
// [0, M], given a = the first edge with c >= p and b = the last edge with
// c <= p.
__device__ inline double quantile_hist_ab(const double *rho, const double *c, const HGrid &g, double p, int a,
                                          int b) {
#pragma clang fp contract(off)
    const int I = g.cells;
    const double M = c[I];
    double L, R;
    if (a == 0) {
        L = hedge(g, 0);
    } else {
        const double t = fmin(fmax((p - c[a - 1]) / rho[a - 1], 0.0), 1.0);
        L = hedge(g, a - 1) + t * g.h;
    }
    if (b == I) {
        R = hedge(g, I);
    } else {
        const double t = fmin(fmax((p - c[b]) / rho[b], 0.0), 1.0);
        R = hedge(g, b) + t * g.h;
    }
    if (p == 0.0) return R;
    if (p == M) return L;
    return 0.5 * (L + R);
}

// Quantile of the histogram rho (cdf c at the I + 1 edges) at level p.
__device__ inline double quantile_hist(const double *rho, const double *c, const HGrid &g, double p) {
    const int I = g.cells;
    p = fmin(fmax(p, 0.0), c[I]);
    return quantile_hist_ab(rho, c, g, p, lower_bound_d(c, I + 1, p), upper_bound_d(c, I + 1, p) - 1);
}

// Quantiles at non-decreasing levels by one thread: the edge indices of
// quantile_hist found once by binary search, then advanced.
struct QuantileWalk {
    int a = -1, u = 0;  // first edge with c >= p, first edge with c > p
    __device__ inline double at(const double *rho, const double *c, const HGrid &g, double p) {
        const int E = g.cells + 1;
        p = fmin(fmax(p, 0.0), c[E - 1]);
        if (a < 0) {
            a = lower_bound_d(c, E, p);
            u = upper_bound_d(c, E, p);
        } else {
            while (a < E && c[a] < p) ++a;
            while (u < E && c[u] <= p) ++u;
        }
        return quantile_hist_ab(rho, c, g, p, a, u - 1);
    }
};

// Left-to-right running sums by one wave (lanes of wave 0 call it):
// out[0] = 0, out[i+1] = out[i] + v(i) for i < n; returns the total to lane 0
// .. 63.  v is read through a functor so that sums of derived values need no
// scratch.
template <class F>
__device__ inline double wave_running_sum(F v, int n, double *out) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    if (out && lane == 0) out[0] = 0.0;
    double carry = 0.0;
    for (int base = 0; base < n; base += 1024) {
        double r[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int idx = base + lane * 16 + i;
            r[i] = idx < n ? v(idx) : 0.0;
        }
        double mine = 0.0;
        for (int l = 0; l < 64; ++l) {
            if (lane == l) {
                double acc = carry;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    if (base + lane * 16 + i < n) acc = acc + r[i];
                    r[i] = acc;
                }
                mine = acc;
            }
            carry = __shfl(mine, l);
        }
        if (out) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int idx = base + lane * 16 + i;
                if (idx < n) out[idx + 1] = r[i];
            }
        }
    }
    return carry;
}

__global__ void zero_u64(uint64_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---------------------------------------------------------------------------
// Restriction.
// ---------------------------------------------------------------------------
// Equal weights: counts per (segment, cell).  Grid (blocks per segment, k).
__global__ void __launch_bounds__(HB_THREADS) hist_count(const double *__restrict__ x, int64_t n, int64_t stride,
                                                         HGrid g, uint64_t *__restrict__ cnt) {
    extern __shared__ uint32_t hc[];
    const int s = blockIdx.y;
    for (int i = threadIdx.x; i < g.cells; i += blockDim.x) hc[i] = 0;
    __syncthreads();
    const double *xs = x + (int64_t)s * stride;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&hc[hcell(g, xs[p])], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < g.cells; i += blockDim.x)
        if (hc[i]) atomicAdd((unsigned long long *)&cnt[(int64_t)s * g.cells + i], (unsigned long long)hc[i]);
}

// Weights: four 32-bit limbs of the 2^-112 fixed-point weight per cell.
__global__ void __launch_bounds__(HB_THREADS) hist_weighted(const double *__restrict__ x, const double *__restrict__ w,
                                                            int64_t n, int64_t stride, HGrid g,
                                                            uint64_t *__restrict__ limbs) {
    extern __shared__ uint64_t hl[];  // [cells][4]
    const int s = blockIdx.y;
    for (int i = threadIdx.x; i < 4 * g.cells; i += blockDim.x) hl[i] = 0;
    __syncthreads();
    const double *xs = x + (int64_t)s * stride;
    const double *ws = w + (int64_t)s * stride;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const u128 q = fix_floor(ws[p], FIX_W);
        const int c = hcell(g, xs[p]);
        const uint64_t lo = (uint64_t)q, hi = (uint64_t)(q >> 64);
        if (lo) {
            atomicAdd((unsigned long long *)&hl[4 * c + 0], (unsigned long long)(lo & 0xFFFFFFFFull));
            atomicAdd((unsigned long long *)&hl[4 * c + 1], (unsigned long long)(lo >> 32));
        }
        if (hi) {
            atomicAdd((unsigned long long *)&hl[4 * c + 2], (unsigned long long)(hi & 0xFFFFFFFFull));
            atomicAdd((unsigned long long *)&hl[4 * c + 3], (unsigned long long)(hi >> 32));
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * g.cells; i += blockDim.x)
        if (hl[i]) atomicAdd((unsigned long long *)&limbs[(int64_t)s * 4 * g.cells + i], (unsigned long long)hl[i]);
}

__global__ void hist_finish_counts(const uint64_t *__restrict__ cnt, int64_t total, double w0, double *__restrict__ rho) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
        rho[i] = (double)cnt[i] * w0;
}

__global__ void hist_finish_limbs(const uint64_t *__restrict__ limbs, int64_t total, double *__restrict__ rho) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t *l = limbs + 4 * i;
        const u128 v = (u128)l[0] + ((u128)l[1] << 32) + ((u128)l[2] << 64) + ((u128)l[3] << 96);
        rho[i] = fix_to_double(v, FIX_W);
    }
}

static HGrid make_hgrid(const pr_grid *grid) {
    HGrid g;
    g.cells = grid->n_cells;
    g.lo = grid->x_lo;
    g.h = (grid->x_hi - grid->x_lo) / grid->n_cells;
    g.inv_h = (double)grid->n_cells / (grid->x_hi - grid->x_lo);
    return g;
}

size_t hist_ws_bytes(int k, int cells) { return sizeof(uint64_t) * 4 * (size_t)k * cells + 256; }

// rho[s][I] of the ensembles x + s*stride (n particles each), s < k.
int hist_restrict(const double *x, const double *w, int64_t n, int64_t stride, int k, const HGrid &g, double *rho,
                  void *ws, hipStream_t st) {
    if (k == 0) return PR_OK;
    uint64_t *acc = (uint64_t *)ws;
    const int64_t words = (int64_t)(w ? 4 : 1) * k * g.cells;
    hipLaunchKernelGGL(zero_u64, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 1024)), dim3(256), 0, st, acc,
                       words);
    PR_LAUNCHED();
    const int per = (int)std::min<int64_t>(std::max<int64_t>((n + 16383) / 16384, 1), 32);
    const dim3 grid((unsigned)per, (unsigned)k);
    if (w) {
        hipLaunchKernelGGL(hist_weighted, grid, dim3(HB_THREADS), sizeof(uint64_t) * 4 * g.cells, st, x, w, n, stride,
                           g, acc);
        PR_LAUNCHED();
        hipLaunchKernelGGL(hist_finish_limbs, dim3((unsigned)std::min<int64_t>(((int64_t)k * g.cells + 255) / 256, 1024)),
                           dim3(256), 0, st, (const uint64_t *)acc, (int64_t)k * g.cells, rho);
    } else {
        hipLaunchKernelGGL(hist_count, grid, dim3(HB_THREADS), sizeof(uint32_t) * g.cells, st, x, n, stride, g, acc);
        PR_LAUNCHED();
        hipLaunchKernelGGL(hist_finish_counts, dim3((unsigned)std::min<int64_t>(((int64_t)k * g.cells + 255) / 256, 1024)),
                           dim3(256), 0, st, (const uint64_t *)acc, (int64_t)k * g.cells, 1.0 / (double)n, rho);
    }
    PR_LAUNCHED();
    return PR_OK;
}

// ---------------------------------------------------------------------------
// Iterators, one slice per workgroup.
// ---------------------------------------------------------------------------
// Scratch of the quantile iterator per slice, in doubles.
__host__ __device__ inline size_t jq_scratch_doubles(int cells) { return (size_t)6 * (cells + 1) + 8; }

template <int KIND>
__global__ void __launch_bounds__(KIND == PR_J_QUANTILE ? JQ_THREADS : HB_THREADS) hist_jump(const double *__restrict__ rc, const double *__restrict__ rf,
                                                        const double *__restrict__ rcs, int64_t in_stride,
                                                        double *__restrict__ out, int64_t out_stride, HGrid g,
                                                        double *__restrict__ scratch) {
#pragma clang fp contract(off)
    const int s = blockIdx.x;
    const int I = g.cells;
    rc += (int64_t)s * in_stride;
    rf += (int64_t)s * in_stride;
    rcs += (int64_t)s * in_stride;
    out += (int64_t)s * out_stride;
    __shared__ double red[4];
    __shared__ int flag;
    if constexpr (KIND == PR_J_ADD || KIND == PR_J_MULT) {
        if (threadIdx.x == 0) flag = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < I; i += blockDim.x) {
            double r;
            if constexpr (KIND == PR_J_ADD) {
                r = rf[i] + (rc[i] - rcs[i]);
                if (r < 0.0) {
                    flag = 1;
                    r = 0.0;
                }
            } else {
                r = rcs[i] > 0.0 ? rf[i] * (rc[i] / rcs[i]) : 0.0;
            }
            out[i] = r;
        }
        __syncthreads();
        const bool rescale = KIND == PR_J_MULT || flag;
        if (rescale) {
            if (threadIdx.x < 64) {
                const double S = wave_running_sum([&](int i) { return out[i]; }, I, nullptr);
                const double M = wave_running_sum([&](int i) { return rf[i]; }, I, nullptr);
                if (threadIdx.x == 0) {
                    red[0] = S;
                    red[1] = M;
                }
            }
            __syncthreads();
            const double S = red[0], M = red[1];
            for (int i = threadIdx.x; i < I; i += blockDim.x) out[i] = S == 0.0 ? rf[i] : out[i] * (M / S);
        }
    } else if constexpr (KIND == PR_J_ROT) {
        const int wave = threadIdx.x >> 6;
        if (wave < 3) {
            double v;
            if (wave == 0) v = wave_running_sum([&](int i) { return sqrt(rf[i] * rcs[i]); }, I, nullptr);
            else if (wave == 1) v = wave_running_sum([&](int i) { return sqrt(rf[i] * rc[i]); }, I, nullptr);
            else v = wave_running_sum([&](int i) { return sqrt(rcs[i] * rc[i]); }, I, nullptr);
            if ((threadIdx.x & 63) == 0) red[wave] = v;
        }
        __syncthreads();
        const double u = red[0], v = red[1], w = red[2];
        const double a = ((u + (2.0 * u) * w) - v) / (1.0 + w);
        const double b = (u + v) / (1.0 + w);
        for (int i = threadIdx.x; i < I; i += blockDim.x) {
            const double t = (a * sqrt(rc[i]) + sqrt(rf[i])) - b * sqrt(rcs[i]);
            out[i] = t * t;
        }
    } else {
        // quantile iterator on the union of the edge levels.  LDS: the three
        // edge cdfs (later the pool sums and the new edge cdf), the corrected
        // quantiles (first the merged levels), the pool counts, the violations
        // and the unique levels.
        extern __shared__ double jq[];
        const int E = I + 1, T3 = 3 * E;
        double *cc = jq, *cf = cc + E, *ccs = cf + E;  // [3E]
        double *qt = jq + T3;                           // [<= 3E]
        int *pC = (int *)(jq + 2 * T3);                 // [<= 3E]
        double *merged = qt;                            // [3E], dead once the levels are unique
        double *lev = (double *)(pC + 2 * T3);          // [3E]
        (void)scratch;
        __shared__ int nU, bad;
        const int wave = threadIdx.x >> 6;
        if (wave == 0) wave_running_sum([&](int i) { return rc[i]; }, I, cc);
        if (wave == 1) wave_running_sum([&](int i) { return rf[i]; }, I, cf);
        if (wave == 2) wave_running_sum([&](int i) { return rcs[i]; }, I, ccs);
        __syncthreads();
        // stable merge by rank: (value, array, index).  Every thread takes a
        // contiguous run of one array's (non-decreasing) values; the ranks in
        // the other two arrays come from one binary search each, then advance.
        {
            const int per = (T3 + JQ_THREADS - 1) / JQ_THREADS;
            const int e0 = threadIdx.x * per, e1 = min(e0 + per, T3);
            int cur = -1, r1 = 0, r2 = 0;
            for (int e = e0; e < e1; ++e) {
                const int arr = e / E, idx = e % E;
                const double *A = arr == 0 ? cc : arr == 1 ? cf : ccs;
                const double *B1 = arr == 0 ? cf : cc;   // first other array
                const double *B2 = arr == 2 ? cf : ccs;  // second other array
                const double v = A[idx];
                // ties: an earlier array's equal values come first
                const bool strict1 = arr == 0;  // B1 later than A: count B1 < v; else B1 <= v
                const bool strict2 = arr != 2;  // B2 later than A: count B2 < v; else B2 <= v
                if (arr != cur) {
                    cur = arr;
                    r1 = strict1 ? lower_bound_d(B1, E, v) : upper_bound_d(B1, E, v);
                    r2 = strict2 ? lower_bound_d(B2, E, v) : upper_bound_d(B2, E, v);
                } else {
                    if (strict1) while (r1 < E && B1[r1] < v) ++r1;
                    else while (r1 < E && B1[r1] <= v) ++r1;
                    if (strict2) while (r2 < E && B2[r2] < v) ++r2;
                    else while (r2 < E && B2[r2] <= v) ++r2;
                }
                merged[idx + r1 + r2] = v;
            }
        }
        __syncthreads();
        // unique levels: compaction of the first of every run of equal values,
        // every thread owning a contiguous chunk of the merged levels
        {
            const int per = (T3 + JQ_THREADS - 1) / JQ_THREADS;
            const int i0 = threadIdx.x * per, i1 = min(i0 + per, T3);
            int cnt = 0;
            for (int i = i0; i < i1; ++i) cnt += (i == 0 || merged[i] != merged[i - 1]) ? 1 : 0;
            __shared__ int wsum[JQ_THREADS / 64];
            const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
            int inc = cnt;
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(inc, off);
                if (lane >= off) inc += t;
            }
            if (lane == 63) wsum[w] = inc;
            __syncthreads();
            int base = inc - cnt;
            for (int k2 = 0; k2 < w; ++k2) base += wsum[k2];
            for (int i = i0; i < i1; ++i)
                if (i == 0 || merged[i] != merged[i - 1]) lev[base++] = merged[i];
            if (threadIdx.x == JQ_THREADS - 1) nU = base;
        }
        __syncthreads();
        const int U = nU;
        {  // every thread a contiguous run of the (increasing) levels
            const int per = (U + JQ_THREADS - 1) / JQ_THREADS;
            const int j0 = threadIdx.x * per, j1 = min(j0 + per, U);
            QuantileWalk wf, wc, wcs;
            for (int j = j0; j < j1; ++j) {
                const double p = lev[j];
                const double qf = wf.at(rf, cf, g, p);
                const double qc = wc.at(rc, cc, g, p);
                const double qcs = wcs.at(rcs, ccs, g, p);
                qt[j] = qf + (qc - qcs);
            }
        }
        __syncthreads();
        // violations qt[j] > qt[j+1], in increasing j, compacted into vio
        int *vio = pC + T3;
        {
            const int per = (U + JQ_THREADS - 1) / JQ_THREADS;
            const int j0 = threadIdx.x * per, j1 = min(j0 + per, U - 1);
            int cnt = 0;
            for (int j = j0; j < j1; ++j) cnt += qt[j] > qt[j + 1] ? 1 : 0;
            __shared__ int vsum[JQ_THREADS / 64];
            const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
            int inc = cnt;
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(inc, off);
                if (lane >= off) inc += t;
            }
            if (lane == 63) vsum[w] = inc;
            __syncthreads();
            int base = inc - cnt;
            for (int k2 = 0; k2 < w; ++k2) base += vsum[k2];
            for (int j = j0; j < j1; ++j)
                if (qt[j] > qt[j + 1]) vio[base++] = j;
            if (threadIdx.x == JQ_THREADS - 1) bad = base;
        }
        __syncthreads();
        if (bad > 0) {  // the cdfs are no longer needed: their LDS holds the pools' sums
            __shared__ PavaChunks pcs;
            pava_block_chunked(qt, U, vio, bad, jq, pC, pcs);
        }
        __syncthreads();
        // cdf at the edges: inf{p : q(p) >= x_i} on the piecewise-linear q
        double *ct = jq;  // [E], over the pool sums
        const int iper = (E + JQ_THREADS - 1) / JQ_THREADS;
        const int i0 = threadIdx.x * iper, i1 = min(i0 + iper, E);
        int jw = -1;  // first level with qt >= x, advanced along the thread's edges
        for (int i = i0; i < i1; ++i) {
            double v;
            if (i == 0) {
                v = 0.0;
            } else if (i == I) {
                v = lev[U - 1];
            } else {
                const double x = hedge(g, i);
                if (jw < 0) jw = lower_bound_d(qt, U, x);
                else while (jw < U && qt[jw] < x) ++jw;
                const int j = jw;
                if (j == 0) v = 0.0;
                else if (j == U) v = lev[U - 1];
                else {
                    const double t = (x - qt[j - 1]) / (qt[j] - qt[j - 1]);
                    v = lev[j - 1] + t * (lev[j] - lev[j - 1]);
                }
            }
            ct[i] = v;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < I; i += blockDim.x) out[i] = ct[i + 1] - ct[i];
    }
}

static size_t jq_lds_bytes(int cells) { return (sizeof(double) * 3 + sizeof(int) * 2) * 3 * (size_t)(cells + 1); }

size_t hist_jump_ws_bytes(int k, int cells) { return sizeof(double) * jq_scratch_doubles(cells) * (size_t)k + 256; }

int hist_jump_launch(int kind, const double *rc, const double *rf, const double *rcs, int64_t in_stride, int k,
                     double *out, int64_t out_stride, const HGrid &g, double *scratch, hipStream_t st) {
    if (k == 0) return PR_OK;
    switch (kind) {
        case PR_J_ADD:
            hipLaunchKernelGGL(hist_jump<PR_J_ADD>, dim3(k), dim3(HB_THREADS), 0, st, rc, rf, rcs, in_stride, out,
                               out_stride, g, scratch);
            break;
        case PR_J_MULT:
            hipLaunchKernelGGL(hist_jump<PR_J_MULT>, dim3(k), dim3(HB_THREADS), 0, st, rc, rf, rcs, in_stride, out,
                               out_stride, g, scratch);
            break;
        case PR_J_ROT:
            hipLaunchKernelGGL(hist_jump<PR_J_ROT>, dim3(k), dim3(HB_THREADS), 0, st, rc, rf, rcs, in_stride, out,
                               out_stride, g, scratch);
            break;
        default:
            hipLaunchKernelGGL(hist_jump<PR_J_QUANTILE>, dim3(k), dim3(JQ_THREADS), jq_lds_bytes(g.cells), st, rc, rf,
                               rcs, in_stride, out, out_stride, g, scratch);
    }
    PR_LAUNCHED();
    return PR_OK;
}

// ---------------------------------------------------------------------------
// Matchings.
// ---------------------------------------------------------------------------
// Per slice tables: cdf of the prior and of the target at the edges, and the
// reweighting ratios rho'_i / rhobar_i (H9 of the design notes).
__global__ void __launch_bounds__(HB_THREADS) match_tables(const double *__restrict__ rt, int64_t t_stride,
                                                           const double *__restrict__ rp, int64_t p_stride, HGrid g,
                                                           int want_ratio, double *__restrict__ tab) {
#pragma clang fp contract(off)
    const int s = blockIdx.x, I = g.cells;
    rt += (int64_t)s * t_stride;
    rp += (int64_t)s * p_stride;
    double *cp = tab + (size_t)s * 3 * (I + 1);
    double *ctg = cp + (I + 1);
    double *ratio = ctg + (I + 1);
    const int wave = threadIdx.x >> 6;
    if (wave == 0) wave_running_sum([&](int i) { return rp[i]; }, I, cp);
    if (wave == 1) wave_running_sum([&](int i) { return rt[i]; }, I, ctg);
    if (want_ratio) {
        // the target mass of cells without prior particles goes to the
        // nearest supported cells, half to each side, in increasing cell order
        __shared__ double r[HB_MAX_CELLS], tg[HB_MAX_CELLS];
        __shared__ int sup[HB_MAX_CELLS], nxt[HB_MAX_CELLS + 1];
        for (int i = threadIdx.x; i < I; i += blockDim.x) {
            sup[i] = rp[i] > 0.0 ? 1 : 0;
            tg[i] = rt[i];
            r[i] = sup[i] ? tg[i] : 0.0;
        }
        __syncthreads();
        if (threadIdx.x == 128) {
            // nxt[i]: first supported cell at or after i (I if none)
            nxt[I] = I;
            for (int i = I - 1; i >= 0; --i) nxt[i] = sup[i] ? i : nxt[i + 1];
            int left = -1;
            for (int i = 0; i < I; ++i) {
                if (sup[i]) {
                    left = i;
                    continue;
                }
                const double m = tg[i];
                if (m == 0.0) continue;
                const int right = nxt[i + 1];
                if (left >= 0 && right < I) {
                    const double half = 0.5 * m;
                    r[left] = r[left] + half;
                    r[right] = r[right] + half;
                } else if (left >= 0) {
                    r[left] = r[left] + m;
                } else if (right < I) {
                    r[right] = r[right] + m;
                }
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < I; i += blockDim.x) ratio[i] = sup[i] ? r[i] / rp[i] : 0.0;
    }
}

static size_t match_tab_doubles(int k, int cells) { return (size_t)3 * (cells + 1) * k; }

struct HMatchArgs {
    const double *rt, *rp;     // [k][I] target and prior histograms (strides)
    int64_t t_stride, p_stride;
    const double *x, *y, *w;   // prior ensemble (strides; w NULL = equal)
    int64_t x_stride;          // elements between slices (0: one prior for all)
    double *xo, *yo, *wo;      // posterior
    int64_t o_stride;
    int64_t n;
    int d;
    const double *tab;         // match_tables output
};

// first index in [lo, hi) with a[i] >= v (hi if none)
__device__ __forceinline__ int lower_bound_range(const double *a, int lo, int hi, double v) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

constexpr int MM_THREADS = 512;

// Fast-marginal matching: X = q_t(cbar(Xbar)).  Grid (tiles, k).
// The level cbar of a particle in prior cell i lies in [cp_i, cp_{i+1}], so
// the first target edge whose cdf reaches it lies between s_i and s_{i+1},
// s_i = the first target edge with cdf >= cp_i (a table in LDS): the search
// covers the few target cells that overlap prior cell i.  When the level
// falls strictly inside a target cell (no target edge has exactly this cdf
// value) the quantile is that cell's linear interpolation, the same value as
// the midpoint rule of the general case; otherwise the general rule runs.
__global__ void __launch_bounds__(MM_THREADS) match_marginal_kernel(HMatchArgs a, HGrid g) {
#pragma clang fp contract(off)
    extern __shared__ double sh[];
    const int s = blockIdx.y, I = g.cells;
    double *rp = sh, *rt = rp + I, *cp = rt + I, *ctg = cp + (I + 1);
    int *st = (int *)(ctg + (I + 1));
    const double *tab = a.tab + (size_t)s * 3 * (I + 1);
    for (int i = threadIdx.x; i < I; i += blockDim.x) {
        rp[i] = a.rp[(int64_t)s * a.p_stride + i];
        rt[i] = a.rt[(int64_t)s * a.t_stride + i];
    }
    for (int i = threadIdx.x; i <= I; i += blockDim.x) {
        cp[i] = tab[i];
        ctg[i] = tab[I + 1 + i];
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= I; i += blockDim.x) st[i] = lower_bound_range(ctg, 0, I + 1, cp[i]);
    __syncthreads();
    const double M = ctg[I];
    const double *x = a.x + (int64_t)s * a.x_stride;
    double *xo = a.xo + (int64_t)s * a.o_stride;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += (int64_t)gridDim.x * blockDim.x) {
        const double xv = x[p];
        const int i = hcell(g, xv);
        const double t = fmin(fmax((xv - hedge(g, i)) / g.h, 0.0), 1.0);
        const double cbar = cp[i] + t * rp[i];
        const double lv = fmin(fmax(cbar, 0.0), M);
        double out;
        if (lv >= cp[i] && lv <= cp[i + 1]) {
            const int e = lower_bound_range(ctg, st[i], min(st[i + 1] + 1, I + 1), lv);
            if (e >= 1 && e <= I && ctg[e] > lv) {
                const double u = fmin(fmax((lv - ctg[e - 1]) / rt[e - 1], 0.0), 1.0);
                out = hedge(g, e - 1) + u * g.h;
            } else {
                out = quantile_hist(rt, ctg, g, lv);
            }
        } else {
            out = quantile_hist(rt, ctg, g, lv);
        }
        xo[p] = out;
    }
}

// Reweighting: W = Wbar * ratio[cell].  Grid (tiles, k).
__global__ void __launch_bounds__(HB_THREADS) reweight_kernel(HMatchArgs a, HGrid g, double w0) {
    const int s = blockIdx.y, I = g.cells;
    const double *ratio = a.tab + (size_t)s * 3 * (I + 1) + 2 * (I + 1);
    const double *x = a.x + (int64_t)s * a.x_stride;
    const double *w = a.w ? a.w + (int64_t)s * a.x_stride : nullptr;
    double *wo = a.wo + (int64_t)s * a.o_stride;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += (int64_t)gridDim.x * blockDim.x)
        wo[p] = (w ? w[p] : w0) * ratio[hcell(g, x[p])];
}

// Inclusive prefix of one u128 per thread over the block, in thread order;
// *total receives the block's sum.
__device__ inline u128 block_inclusive_u128(u128 v, u128 *total) {
    __shared__ uint64_t wt[16][2];  // blocks of up to 1024 threads
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    u128 inc = v;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long lo = __shfl_up((unsigned long long)(uint64_t)inc, off);
        const unsigned long long hi = __shfl_up((unsigned long long)(uint64_t)(inc >> 64), off);
        if (lane >= off) inc += ((u128)hi << 64) | (u128)lo;
    }
    if (lane == 63) {
        wt[w][0] = (uint64_t)inc;
        wt[w][1] = (uint64_t)(inc >> 64);
    }
    __syncthreads();
    u128 pre = 0, tot = 0;
    for (int k2 = 0; k2 < (int)(blockDim.x >> 6); ++k2) {
        const u128 t = (u128)wt[k2][0] | ((u128)wt[k2][1] << 64);
        if (k2 < w) pre += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return pre + inc;
}

// The reweighting ratios of slice s into LDS.
__device__ inline void load_ratio(const HMatchArgs &a, const HGrid &g, int s, double *r) {
    const int I = g.cells;
    const double *ratio = a.tab + (size_t)s * 3 * (I + 1) + 2 * (I + 1);
    for (int i = threadIdx.x; i < I; i += blockDim.x) r[i] = ratio[i];
    __syncthreads();
}

// Resampling, pass 1: exact tile sums of the fixed-point weights.  Grid
// (tiles, k); a tile is HB_TILE particles, row i of a tile the particles
// tile * HB_TILE + i * HB_THREADS + thread.
__global__ void __launch_bounds__(HB_THREADS) resample_tile_sums(HMatchArgs a, HGrid g, double w0, int ntile,
                                                                 uint64_t *__restrict__ tsum) {
    __shared__ double r[HB_MAX_CELLS];
    const int s = blockIdx.y;
    load_ratio(a, g, s, r);
    const double *x = a.x + (int64_t)s * a.x_stride;
    const double *w = a.w ? a.w + (int64_t)s * a.x_stride : nullptr;
    const int64_t p0 = (int64_t)blockIdx.x * HB_TILE + threadIdx.x;
    u128 acc = 0;
    for (int i = 0; i < HB_ITEMS; ++i) {
        const int64_t p = p0 + (int64_t)i * HB_THREADS;
        if (p < a.n) acc += (u128)fix_weight((w ? w[p] : w0) * r[hcell(g, x[p])]);
    }
    u128 tot;
    (void)block_inclusive_u128(acc, &tot);
    if (threadIdx.x == 0) {
        uint64_t *o = tsum + 2 * ((int64_t)s * ntile + blockIdx.x);
        o[0] = (uint64_t)tot;
        o[1] = (uint64_t)(tot >> 64);
    }
}

// Pass 2: exclusive prefix over the tiles of every slice, and the total.
// One block per slice, HB_THREADS tiles at a time.
__global__ void __launch_bounds__(HB_THREADS) resample_tile_scan(uint64_t *__restrict__ tsum, int ntile, int64_t P,
                                                                 uint64_t *__restrict__ total) {
    const int s = blockIdx.x;
    uint64_t *t = tsum + 2 * (int64_t)s * ntile;
    u128 run = 0;
    for (int c0 = 0; c0 < ntile; c0 += HB_THREADS) {
        const int i = c0 + (int)threadIdx.x;
        const u128 v = i < ntile ? ((u128)t[2 * i] | ((u128)t[2 * i + 1] << 64)) : (u128)0;
        u128 chunk;
        const u128 inc = block_inclusive_u128(v, &chunk);
        if (i < ntile) {
            const u128 ex = run + (inc - v);
            t[2 * i] = (uint64_t)ex;
            t[2 * i + 1] = (uint64_t)(ex >> 64);
        }
        run += chunk;
    }
    if (threadIdx.x == 0) {
        total[5 * s] = (uint64_t)run;
        total[5 * s + 1] = (uint64_t)(run >> 64);
        const u128 qT = udiv128_32(run, (uint32_t)P);
        total[5 * s + 2] = (uint64_t)qT;
        total[5 * s + 3] = (uint64_t)(qT >> 64);
        total[5 * s + 4] = (uint64_t)(run - qT * (u128)P);
    }
}

// first slot j in [0, P] with U_j >= C (U is non-decreasing in j), from the
// estimate j = C P / T
__device__ inline int64_t first_slot_at(u128 C, u128 T, double Td, const SlotConst &sc, uint32_t P, Key key,
                                        uint32_t inst, uint32_t tpnt, int det) {
    if (C >= T) return (int64_t)P;
    int64_t j = (int64_t)(fix_to_double(C, 0) / Td * (double)P);
    j = j < 0 ? 0 : (j > (int64_t)P ? (int64_t)P : j);
    while (j > 0 && slot_level((uint64_t)(j - 1), slot_draw(key, inst, (uint32_t)(j - 1), tpnt, det), sc, P) >= C) --j;
    while (j < (int64_t)P && slot_level((uint64_t)j, slot_draw(key, inst, (uint32_t)j, tpnt, det), sc, P) < C) ++j;
    return j;
}

constexpr int RS_THREADS = 512, RS_ITEMS = HB_TILE / RS_THREADS;

// Pass 3: the slots of a tile.  The block lays the cumulative weights of its
// particles out in LDS, finds the slots j whose level U_j falls inside the
// tile's weight range, and gives each of them the particle p with
// C_p <= U_j < C_{p+1} (the first whose inclusive sum exceeds U_j).
__global__ void __launch_bounds__(RS_THREADS) resample_slots_kernel(HMatchArgs a, HGrid g, double w0, int ntile,
                                                                    const uint64_t *__restrict__ tsum,
                                                                    const uint64_t *__restrict__ total, Key key,
                                                                    uint32_t inst, int t_first, int det) {
    __shared__ double r[HB_MAX_CELLS];
    __shared__ uint64_t cum[HB_TILE][2];  // inclusive cumulative weight of every particle of the tile
    __shared__ int64_t jr[2];
    __shared__ int sidx[HB_TILE];  // particle of every slot of a batch
    const int s = blockIdx.y;
    load_ratio(a, g, s, r);
    const double *x = a.x + (int64_t)s * a.x_stride;
    const double *w = a.w ? a.w + (int64_t)s * a.x_stride : nullptr;
    const double *y = a.y + (int64_t)s * a.x_stride * a.d;
    double *xo = a.xo + (int64_t)s * a.o_stride;
    double *yo = a.yo + (int64_t)s * a.o_stride * a.d;
    double *wo = a.wo + (int64_t)s * a.o_stride;
    const uint32_t P = (uint32_t)a.n;
    const u128 T = (u128)total[5 * s] | ((u128)total[5 * s + 1] << 64);
    SlotConst sc;
    sc.qT = (u128)total[5 * s + 2] | ((u128)total[5 * s + 3] << 64);
    sc.rT = total[5 * s + 4];
    sc.inv_p = 1.0 / (double)P;
    const double Td = fix_to_double(T, 0);
    const uint64_t *tp = tsum + 2 * ((int64_t)s * ntile + blockIdx.x);
    const u128 start = (u128)tp[0] | ((u128)tp[1] << 64);
    const uint32_t tpnt = (uint32_t)(t_first + s);
    const int64_t t0 = (int64_t)blockIdx.x * HB_TILE;
    const int np = (int)((a.n - t0) < HB_TILE ? (a.n - t0) : HB_TILE);
    // every thread sums RS_ITEMS consecutive particles, one block scan of
    // the thread sums places them (integer sums: the order is immaterial)
    u128 c = 0, own[RS_ITEMS];
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int idx = (int)threadIdx.x * RS_ITEMS + i;
        const int64_t p = t0 + idx;
        c += (u128)(idx < np ? fix_weight((w ? w[p] : w0) * r[hcell(g, x[p])]) : 0ull);
        own[i] = c;
    }
    u128 tile_total;
    const u128 before = start + (block_inclusive_u128(c, &tile_total) - c);
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int idx = (int)threadIdx.x * RS_ITEMS + i;
        const u128 v = before + own[i];
        cum[idx][0] = (uint64_t)v;
        cum[idx][1] = (uint64_t)(v >> 64);
    }
    const u128 row0 = start + tile_total;
    if (threadIdx.x == 0) jr[0] = first_slot_at(start, T, Td, sc, P, key, inst, tpnt, det);
    if (threadIdx.x == 64)
        jr[1] = (int)blockIdx.x == ntile - 1 ? (int64_t)P : first_slot_at(row0, T, Td, sc, P, key, inst, tpnt, det);
    __syncthreads();
    // slots in batches of HB_TILE: every thread finds the particles of a
    // contiguous run of slots (one binary search, then a walk: U_j grows
    // with j), then the block copies them with coalesced stores
    for (int64_t jb = jr[0]; jb < jr[1]; jb += HB_TILE) {
        const int nb = (int)((jr[1] - jb) < HB_TILE ? (jr[1] - jb) : HB_TILE);
        const int per = (nb + RS_THREADS - 1) / RS_THREADS;
        const int s0 = (int)threadIdx.x * per, s1 = min(s0 + per, nb);
        int idx = -1;  // first idx with cum[idx] > U (the last particle takes the rest)
        for (int t = s0; t < s1; ++t) {
            const int64_t j = jb + t;
            const u128 U = slot_level((uint64_t)j, slot_draw(key, inst, (uint32_t)j, tpnt, det), sc, P);
            if (idx < 0) {
                int lo = 0, hi = np - 1;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    const u128 cm = (u128)cum[mid][0] | ((u128)cum[mid][1] << 64);
                    if (cm > U) hi = mid;
                    else lo = mid + 1;
                }
                idx = lo;
            } else {
                while (idx < np - 1 && !(((u128)cum[idx][0] | ((u128)cum[idx][1] << 64)) > U)) ++idx;
            }
            sidx[t] = idx;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < nb; t += RS_THREADS) {
            const int64_t j = jb + t, p = t0 + sidx[t];
            xo[j] = x[p];
            for (int c = 0; c < a.d; ++c) yo[(int64_t)c * a.n + j] = y[(int64_t)c * a.n + p];
            wo[j] = w0;
        }
        __syncthreads();
    }
}

size_t hist_match_ws_bytes(int64_t n, int k, int cells) {
    const int64_t ntile = (n + HB_TILE - 1) / HB_TILE;
    return sizeof(double) * match_tab_doubles(k, cells) + sizeof(uint64_t) * (2 * (size_t)ntile * k + 5 * (size_t)k) + 512;
}

int hist_match(int kind, const HMatchArgs &a0, int k, const HGrid &g, Key key, uint32_t inst, int t_first, void *ws,
               hipStream_t st) {
    if (k == 0 || a0.n == 0) return PR_OK;
    HMatchArgs a = a0;
    double *tab = (double *)ws;
    a.tab = tab;
    const double w0 = 1.0 / (double)a.n;
    hipLaunchKernelGGL(match_tables, dim3(k), dim3(HB_THREADS), 0, st, a.rt, a.t_stride, a.rp, a.p_stride, g,
                       kind == PR_M_MARGINAL ? 0 : 1, tab);
    PR_LAUNCHED();
    const int per = (int)std::min<int64_t>(std::max<int64_t>((a.n + 4095) / 4096, 1), 256);
    const dim3 grid((unsigned)per, (unsigned)k);
    if (kind == PR_M_MARGINAL) {
        hipLaunchKernelGGL(match_marginal_kernel, grid, dim3(MM_THREADS),
                           sizeof(double) * (4 * g.cells + 2) + sizeof(int) * (g.cells + 1), st, a, g);
        PR_LAUNCHED();
        return PR_OK;
    }
    if (kind == PR_M_REWEIGHT) {
        hipLaunchKernelGGL(reweight_kernel, grid, dim3(HB_THREADS), 0, st, a, g, w0);
        PR_LAUNCHED();
        return PR_OK;
    }
    const int ntile = (int)((a.n + HB_TILE - 1) / HB_TILE);
    uint64_t *tsum = (uint64_t *)(tab + match_tab_doubles(k, g.cells));
    uint64_t *total = tsum + 2 * (size_t)ntile * k;
    const dim3 tgrid((unsigned)ntile, (unsigned)k);
    hipLaunchKernelGGL(resample_tile_sums, tgrid, dim3(HB_THREADS), 0, st, a, g, w0, ntile, tsum);
    PR_LAUNCHED();
    hipLaunchKernelGGL(resample_tile_scan, dim3(k), dim3(HB_THREADS), 0, st, tsum, ntile, a.n, total);
    PR_LAUNCHED();
    hipLaunchKernelGGL(resample_slots_kernel, tgrid, dim3(RS_THREADS), 0, st, a, g, w0, ntile, (const uint64_t *)tsum,
                       (const uint64_t *)total, key, inst, t_first, kind == PR_M_RESAMPLE_DET ? 1 : 0);
    PR_LAUNCHED();
    return PR_OK;
}

// ---------------------------------------------------------------------------
// Driver.
// ---------------------------------------------------------------------------
__global__ void hist_error_kernel(const double *__restrict__ rho, const double *__restrict__ ref, int K, int I,
                                  double *__restrict__ err) {
    __shared__ double e[1024];
    for (int t = threadIdx.x; t <= K; t += blockDim.x) {
        double s = 0.0;
        for (int i = 0; i < I; ++i) {
            const double d = rho[(size_t)t * I + i] - ref[(size_t)t * I + i];
            s += d * d;
        }
        e[t] = sqrt(s);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int t = 0; t <= K; ++t) m = e[t] > m ? e[t] : m;
        err[0] = e[K];
        err[1] = m;
    }
}

struct HistPR {
    bool chem_model = false;  // the chemical-reaction system instead of sde
    pr_chem chem{};
    pr_sde sde;
    pr_schedule sch;
    pr_grid grid;
    HGrid g;
    uint64_t seed;
    uint32_t inst;
    int64_t n;
    int K, D, I, jkind, mkind, flags;
    bool weighted;
    Coarse *coarse = nullptr;
    double *a = nullptr;
    double *x[3] = {}, *y[3] = {}, *w[3] = {};  // [K+1][n], [K+1][D][n], [K+1][n]
    double *rho = nullptr, *rho_new = nullptr;  // [K+1][I] coarse-level states
    double *rho_f = nullptr, *rho_r = nullptr, *rho_cs = nullptr, *rho_c = nullptr;
    double *err = nullptr;
    void *hws = nullptr, *jws = nullptr, *mws = nullptr;
    int cur = 0, k = 0;
    hipEvent_t ev[PR_PH_COUNT + 1] = {};
    double ph_ms[PR_PH_COUNT] = {};
    int timed = 0;

    double *xs(int b, int t) const { return x[b] + (size_t)t * n; }
    double *ys(int b, int t) const { return y[b] + (size_t)t * D * n; }
    double *wsl(int b, int t) const { return weighted ? w[b] + (size_t)t * n : nullptr; }
    double *row(double *base, int t) const { return base + (size_t)t * I; }
};

static void hist_free(HistPR *h) {
    if (!h) return;
    if (h->coarse) coarse_free(h->coarse);
    void *ptrs[] = {h->a, h->x[0], h->x[1], h->x[2], h->y[0], h->y[1], h->y[2], h->w[0], h->w[1], h->w[2],
                    h->rho, h->rho_new, h->rho_f, h->rho_r, h->rho_cs, h->rho_c, h->err, h->hws, h->jws, h->mws};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (hipEvent_t e : h->ev)
        if (e) (void)hipEventDestroy(e);
    delete h;
}

#define HPR_ALLOC(ptr, bytes)                                                 \
    do {                                                                      \
        if (hipMalloc((void **)&(ptr), (bytes)) != hipSuccess) {              \
            set_error("device allocation of %zu bytes failed", (size_t)(bytes)); \
            hist_free(h);                                                     \
            return PR_E_NOMEM;                                                \
        }                                                                     \
    } while (0)

#define HPR_TRY(expr)                \
    do {                             \
        int s_ = (expr);             \
        if (s_ != PR_OK) {           \
            hist_free(h);            \
            return s_;               \
        }                            \
    } while (0)

static int copy_d(void *dst, const void *src, size_t bytes, hipStream_t st) {
    if (bytes == 0 || dst == src) return PR_OK;
    PR_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
    return PR_OK;
}

__global__ void fill_f64(double *p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Matching of the slices t = 1..K: targets rho_t rows 1..K, priors given by
// buffer pb (slot t, or slot 0 for every slice when prior0), prior
// histograms rho_p rows (1..K or row 0), output into buffer ob.
static int hist_match_states(HistPR *h, const double *rho_t, const double *rho_p, bool prior0, int pb, int ob,
                             hipStream_t st) {
    const int K = h->K;
    const int64_t n = h->n;
    const bool resample = h->mkind == PR_M_RESAMPLE || h->mkind == PR_M_RESAMPLE_DET;
    const int ps = prior0 ? 0 : 1;
    HMatchArgs a{};
    a.rt = rho_t;
    a.t_stride = h->I;
    a.rp = rho_p;
    a.p_stride = prior0 ? 0 : h->I;
    a.x = h->xs(pb, ps);
    a.y = h->ys(pb, ps);
    a.w = h->wsl(pb, ps);
    a.x_stride = prior0 ? 0 : n;
    a.xo = h->xs(ob, 1);
    a.yo = h->ys(ob, 1);
    a.wo = h->weighted ? h->wsl(ob, 1) : (resample ? h->w[ob] + n : nullptr);
    a.o_stride = n;
    a.n = n;
    a.d = h->D;
    if (h->mkind == PR_M_MARGINAL) {
        if (prior0) {
            // every slice starts from the prior's fast variables and weights
            for (int t = 1; t <= K; ++t) {
                PR_CHECK(copy_d(h->ys(ob, t), h->ys(pb, 0), sizeof(double) * h->D * n, st));
                if (h->weighted) PR_CHECK(copy_d(h->wsl(ob, t), h->wsl(pb, 0), sizeof(double) * n, st));
            }
        }
    } else if (h->mkind == PR_M_REWEIGHT) {
        if (prior0 || pb != ob)
            for (int t = 1; t <= K; ++t) {
                PR_CHECK(copy_d(h->xs(ob, t), h->xs(pb, prior0 ? 0 : t), sizeof(double) * n, st));
                PR_CHECK(copy_d(h->ys(ob, t), h->ys(pb, prior0 ? 0 : t), sizeof(double) * h->D * n, st));
            }
    }
    return hist_match(h->mkind, a, K, h->g, make_key(h->seed), h->inst, 1, h->mws, st);
}

// Exactly one of sde_in and chem is non-NULL.
int hist_parareal_create(const pr_sde *sde_in, const pr_chem *chem, const pr_schedule *sch, const pr_grid *grid,
                         uint64_t seed, uint32_t inst, int64_t n, int jkind, int mkind, int flags, hipStream_t st,
                         HistPR **out) {
    HistPR *h = new HistPR();
    pr_sde one{};
    one.d_fast = 1;
    one.precision = PR_F64;
    if (chem) {
        h->chem_model = true;
        h->chem = *chem;
        sde_in = &one;
    }
    h->sde = *sde_in;
    h->sch = *sch;
    h->grid = *grid;
    h->g = make_hgrid(grid);
    h->seed = seed;
    h->inst = inst;
    h->n = n;
    h->K = sch->n_slices;
    h->D = sde_in->d_fast;
    h->I = grid->n_cells;
    h->jkind = jkind;
    h->mkind = mkind;
    h->flags = flags;
    h->weighted = mkind == PR_M_REWEIGHT;
    const int K = h->K, D = h->D, I = h->I;
    const bool resample = mkind == PR_M_RESAMPLE || mkind == PR_M_RESAMPLE_DET;
    if (sde_in->a) {
        HPR_ALLOC(h->a, sizeof(double) * D);
        HPR_TRY(copy_d(h->a, sde_in->a, sizeof(double) * D, st));
        h->sde.a = h->a;
    }
    const size_t xb = sizeof(double) * (size_t)(K + 1) * n;
    const int nbuf = resample ? 3 : 2;
    for (int b = 0; b < nbuf; ++b) {
        HPR_ALLOC(h->x[b], xb);
        HPR_ALLOC(h->y[b], xb * D);
        if (h->weighted || resample) HPR_ALLOC(h->w[b], xb);
    }
    const size_t rb = sizeof(double) * (size_t)(K + 1) * I;
    HPR_ALLOC(h->rho, rb);
    HPR_ALLOC(h->rho_new, rb);
    HPR_ALLOC(h->rho_f, rb);
    HPR_ALLOC(h->rho_r, rb);
    HPR_ALLOC(h->rho_cs, rb);
    HPR_ALLOC(h->rho_c, sizeof(double) * I);
    HPR_ALLOC(h->err, sizeof(double) * 2);
    HPR_ALLOC(h->hws, hist_ws_bytes(K + 1, I));
    HPR_ALLOC(h->jws, hist_jump_ws_bytes(1, I));
    HPR_ALLOC(h->mws, hist_match_ws_bytes(n, K, I));
    if (h->chem_model)
        HPR_TRY(chem_coarse_create(&h->chem, sch, grid, st, &h->coarse));
    else
        HPR_TRY(coarse_create(&h->sde, sch, grid, st, &h->coarse));
    if (flags & PR_PROFILE)
        for (hipEvent_t &e : h->ev) HPR_TRY(hipEventCreate(&e) == hipSuccess ? PR_OK : PR_E_HIP);

    // initial ensemble (and equal weights) in slot 0 of every buffer
    if (h->chem_model)
        HPR_TRY(chem_init_ensemble(&h->chem, seed, inst, n, h->xs(0, 0), h->ys(0, 0), st));
    else
        HPR_TRY(init_ensemble(&h->sde, seed, inst, n, h->xs(0, 0), h->ys(0, 0), st));
    for (int b = 0; b < nbuf; ++b) {
        if (h->w[b]) {
            hipLaunchKernelGGL(fill_f64, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0, st,
                               h->w[b], n, 1.0 / (double)n);
            HPR_TRY(hipGetLastError() == hipSuccess ? PR_OK : PR_E_HIP);
        }
        if (b > 0) {
            HPR_TRY(copy_d(h->xs(b, 0), h->xs(0, 0), sizeof(double) * n, st));
            HPR_TRY(copy_d(h->ys(b, 0), h->ys(0, 0), sizeof(double) * D * n, st));
        }
    }
    // zeroth iteration: rho^0 = R(X0), rho^{n+1} = C_n(rho^n), X^n = M(rho^n; X0)
    HPR_TRY(hist_restrict(h->xs(0, 0), h->wsl(0, 0), n, n, 1, h->g, h->rho, h->hws, st));
    for (int t = 0; t < K; ++t) HPR_TRY(coarse_apply(h->coarse, t, 1, h->row(h->rho, t), h->row(h->rho, t + 1), st));
    HPR_TRY(hist_match_states(h, h->row(h->rho, 1), h->rho, true, 0, 0, st));
    if (hipStreamSynchronize(st) != hipSuccess) {
        set_error("zeroth iteration failed on the device");
        hist_free(h);
        return PR_E_HIP;
    }
    *out = h;
    return PR_OK;
}

int hist_parareal_iterate(HistPR *h, int n_iter, const double *rho_ref, double *err_out, hipStream_t st) {
    const int K = h->K, I = h->I;
    const int64_t n = h->n;
    const bool prof = (h->flags & PR_PROFILE) != 0;
    const bool resample = h->mkind == PR_M_RESAMPLE || h->mkind == PR_M_RESAMPLE_DET;
    auto mark = [&](int i) -> int {
        if (prof) PR_HIP(hipEventRecord(h->ev[i], st));
        return PR_OK;
    };
    for (int it = 0; it < n_iter; ++it) {
        const int c = h->cur, nx = (c + 1) % (resample ? 3 : 2), sp = resample ? (c + 2) % 3 : -1;
        PR_CHECK(mark(0));
        // 1. fine: Xbar^{t+1} = F_t(X_k^t) into buffer nx; the weights ride along
        if (h->chem_model)
            PR_CHECK(chem_fine_propagate(&h->chem, &h->sch, h->seed, h->inst, n, 0, K, h->xs(c, 0), h->ys(c, 0),
                                         h->xs(nx, 1), h->ys(nx, 1), st));
        else
            PR_CHECK(fine_propagate(&h->sde, &h->sch, h->seed, h->inst, n, 0, K, h->xs(c, 0), h->ys(c, 0),
                                    h->xs(nx, 1), h->ys(nx, 1), st));
        if (h->weighted) PR_CHECK(copy_d(h->wsl(nx, 1), h->wsl(c, 0), sizeof(double) * K * n, st));
        PR_CHECK(mark(1));
        // 2. restriction of the fine results
        PR_CHECK(hist_restrict(h->xs(nx, 1), h->wsl(nx, 1), n, n, K, h->g, h->row(h->rho_f, 1), h->hws, st));
        PR_CHECK(mark(2));
        // 3. coarse propagation of the restricted current states
        const double *rin = h->rho;
        if (!(h->flags & PR_REUSE_COARSE)) {
            PR_CHECK(hist_restrict(h->xs(c, 0), h->wsl(c, 0), n, n, K, h->g, h->rho_r, h->hws, st));
            rin = h->rho_r;
        }
        PR_CHECK(coarse_apply(h->coarse, 0, K, rin, h->row(h->rho_cs, 1), st));
        PR_CHECK(mark(3));
        // 4. serial chain: rho^{t+1} = J(C_t(rho^t), rho_f^{t+1}, rho_cs^{t+1})
        PR_CHECK(copy_d(h->rho_new, h->rho, sizeof(double) * I, st));
        for (int t = 0; t < K; ++t) {
            PR_CHECK(coarse_apply(h->coarse, t, 1, h->row(h->rho_new, t), h->rho_c, st));
            PR_CHECK(hist_jump_launch(h->jkind, h->rho_c, h->row(h->rho_f, t + 1), h->row(h->rho_cs, t + 1), 0, 1,
                                      h->row(h->rho_new, t + 1), 0, h->g, (double *)h->jws, st));
        }
        PR_CHECK(mark(4));
        // 5. matching against the fine results
        const int ob = resample ? sp : nx;
        PR_CHECK(hist_match_states(h, h->row(h->rho_new, 1), h->row(h->rho_f, 1), false, nx, ob, st));
        std::swap(h->rho, h->rho_new);
        h->cur = ob;
        PR_CHECK(mark(5));
        // 6. histograms of the new states and their error
        if (rho_ref || err_out) {
            PR_CHECK(hist_restrict(h->xs(ob, 0), h->wsl(ob, 0), n, n, K + 1, h->g, h->rho_r, h->hws, st));
            if (rho_ref) {
                hipLaunchKernelGGL(hist_error_kernel, dim3(1), dim3(256), 0, st, (const double *)h->rho_r, rho_ref, K,
                                   I, h->err);
                PR_LAUNCHED();
            }
        }
        PR_CHECK(mark(6));
        h->k += 1;
        if (err_out && rho_ref) {
            PR_HIP(hipMemcpyAsync(err_out + 2 * it, h->err, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
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

// ---------------------------------------------------------------------------
// Deterministic parareal on cell masses (the linear-advection study): F and C
// are two coarse handles, restriction and matching the identity.
// ---------------------------------------------------------------------------
struct FpPR {
    const Coarse *fine = nullptr, *coarse = nullptr;
    HGrid g;
    int K = 0, I = 0, jkind = 0, k = 0;
    double *rho = nullptr, *rho_new = nullptr;  // [K+1][I]
    double *rho_f = nullptr, *rho_cs = nullptr; // [K+1][I], rows 1..K used
    double *rho_c = nullptr;                    // [I]
    double *err = nullptr;                      // [2]
    void *jws = nullptr;
    double *row(double *b, int t) const { return b + (size_t)t * I; }
};

static void fp_free(FpPR *h) {
    if (!h) return;
    void *ptrs[] = {h->rho, h->rho_new, h->rho_f, h->rho_cs, h->rho_c, h->err, h->jws};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete h;
}

int fp_parareal_create(const Coarse *fine, const Coarse *coarse, const pr_grid *grid, const double *rho0, int jkind,
                       hipStream_t st, FpPR **out) {
    FpPR *h = new FpPR();
    h->fine = fine;
    h->coarse = coarse;
    h->g = make_hgrid(grid);
    h->K = coarse_n_slices(coarse);
    h->I = grid->n_cells;
    h->jkind = jkind;
    const size_t rb = sizeof(double) * (size_t)(h->K + 1) * h->I;
    auto fail = [&](int code, const char *what) {
        set_error("%s", what);
        fp_free(h);
        return code;
    };
    if (hipMalloc(&h->rho, rb) != hipSuccess || hipMalloc(&h->rho_new, rb) != hipSuccess ||
        hipMalloc(&h->rho_f, rb) != hipSuccess || hipMalloc(&h->rho_cs, rb) != hipSuccess ||
        hipMalloc(&h->rho_c, sizeof(double) * h->I) != hipSuccess || hipMalloc(&h->err, 2 * sizeof(double)) != hipSuccess ||
        hipMalloc(&h->jws, hist_jump_ws_bytes(1, h->I)) != hipSuccess)
        return fail(PR_E_NOMEM, "device allocation of the parareal state failed");
    if (copy_d(h->rho, rho0, sizeof(double) * h->I, st) != PR_OK) return fail(PR_E_HIP, "copy of rho0 failed");
    for (int t = 0; t < h->K; ++t)
        if (coarse_apply(coarse, t, 1, h->row(h->rho, t), h->row(h->rho, t + 1), st) != PR_OK)
            return fail(PR_E_HIP, "zeroth iteration failed");
    if (hipStreamSynchronize(st) != hipSuccess) return fail(PR_E_HIP, "zeroth iteration failed on the device");
    *out = h;
    return PR_OK;
}

int fp_parareal_iterate(FpPR *h, int n_iter, const double *rho_ref, double *err_out, hipStream_t st) {
    const int K = h->K, I = h->I;
    for (int it = 0; it < n_iter; ++it) {
        // fine and coarse propagation of the current states, all slices at once
        PR_CHECK(coarse_apply(h->fine, 0, K, h->rho, h->row(h->rho_f, 1), st));
        PR_CHECK(coarse_apply(h->coarse, 0, K, h->rho, h->row(h->rho_cs, 1), st));
        // serial chain
        PR_CHECK(copy_d(h->rho_new, h->rho, sizeof(double) * I, st));
        for (int t = 0; t < K; ++t) {
            PR_CHECK(coarse_apply(h->coarse, t, 1, h->row(h->rho_new, t), h->rho_c, st));
            PR_CHECK(hist_jump_launch(h->jkind, h->rho_c, h->row(h->rho_f, t + 1), h->row(h->rho_cs, t + 1), 0, 1,
                                      h->row(h->rho_new, t + 1), 0, h->g, (double *)h->jws, st));
        }
        std::swap(h->rho, h->rho_new);
        h->k += 1;
        if (rho_ref) {
            hipLaunchKernelGGL(hist_error_kernel, dim3(1), dim3(256), 0, st, (const double *)h->rho, rho_ref, K, I,
                               h->err);
            PR_LAUNCHED();
            if (err_out) {
                PR_HIP(hipMemcpyAsync(err_out + 2 * it, h->err, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
                PR_HIP(hipStreamSynchronize(st));
            }
        }
    }
    return PR_OK;
}

}  // namespace pr

using namespace pr;

static int check_hist_grid(const pr_grid *grid) {
    PR_CHECK(check_grid(grid));
    PR_REQUIRE(grid->n_cells <= HB_MAX_CELLS, "histogram states serve at most %d cells", HB_MAX_CELLS);
    return PR_OK;
}

extern "C" size_t pr_hist_workspace_size(int k, int n_cells) { return hist_ws_bytes(k, n_cells); }

extern "C" int pr_hist_restrict(const double *x, const double *w, int64_t n, int k, const pr_grid *grid, double *rho,
                                void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    PR_CHECK(check_hist_grid(grid));
    PR_REQUIRE(n >= 1 && n <= 0xFFFFFFFFll && k >= 0 && k <= 65535, "need 1 <= n < 2^32 and 0 <= k <= 65535");
    PR_REQUIRE(k == 0 || (x && rho && ws), "x, rho and ws must be non-NULL");
    PR_REQUIRE(ws_bytes >= hist_ws_bytes(k, grid->n_cells), "workspace too small: %zu < %zu", ws_bytes,
               hist_ws_bytes(k, grid->n_cells));
    return hist_restrict(x, w, n, n, k, make_hgrid(grid), rho, ws, as_stream(stream));
}

extern "C" size_t pr_hist_jump_workspace_size(int k, int n_cells) { return hist_jump_ws_bytes(k, n_cells); }

extern "C" int pr_hist_jump(int kind, const double *rho_c, const double *rho_f, const double *rho_cs, int k,
                            const pr_grid *grid, double *rho_out, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    PR_CHECK(check_hist_grid(grid));
    PR_REQUIRE(kind >= PR_J_ADD && kind <= PR_J_QUANTILE, "unknown iterator %d", kind);
    PR_REQUIRE(k >= 0 && k <= 65535, "need 0 <= k <= 65535");
    PR_REQUIRE(k == 0 || (rho_c && rho_f && rho_cs && rho_out), "histograms must be non-NULL");
    PR_REQUIRE(kind != PR_J_QUANTILE || k == 0 || (ws && ws_bytes >= hist_jump_ws_bytes(k, grid->n_cells)),
               "the quantile iterator needs %zu bytes of workspace", hist_jump_ws_bytes(k, grid->n_cells));
    const int I = grid->n_cells;
    return hist_jump_launch(kind, rho_c, rho_f, rho_cs, I, k, rho_out, I, make_hgrid(grid), (double *)ws,
                            as_stream(stream));
}

extern "C" size_t pr_hist_match_workspace_size(int64_t n, int k, int n_cells) {
    return hist_match_ws_bytes(n, k, n_cells);
}

extern "C" int pr_hist_match(int kind, const double *rho_t, const double *rho_p, int64_t n, int k, int d,
                             const pr_grid *grid, const double *x, const double *y, const double *w, int64_t prior_stride,
                             double *x_out, double *y_out, double *w_out, uint64_t seed, uint32_t instance,
                             int t_first, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    PR_CHECK(check_hist_grid(grid));
    PR_REQUIRE(kind >= PR_M_MARGINAL && kind <= PR_M_RESAMPLE_DET, "unknown matching %d", kind);
    PR_REQUIRE(n >= 1 && n <= 0xFFFFFFFFll && k >= 0 && k <= 65535, "need 1 <= n < 2^32 and 0 <= k <= 65535");
    PR_REQUIRE(valid_d(d), "d = %d not served", d);
    PR_REQUIRE(prior_stride == 0 || prior_stride == n, "prior_stride must be 0 (one prior) or n");
    PR_REQUIRE(t_first >= 0 && t_first + k <= 65536, "time points must stay below 65536");
    PR_REQUIRE(k == 0 || (rho_t && rho_p && x && ws), "histograms, x and ws must be non-NULL");
    PR_REQUIRE(kind == PR_M_MARGINAL || k == 0 || w_out, "w_out must be non-NULL for the conditional matchings");
    PR_REQUIRE(kind == PR_M_MARGINAL || kind == PR_M_REWEIGHT || k == 0 || (y && y_out && x_out),
               "resampling needs x, y and their outputs");
    PR_REQUIRE(kind != PR_M_MARGINAL || k == 0 || x_out, "x_out must be non-NULL");
    PR_REQUIRE(!(kind == PR_M_RESAMPLE || kind == PR_M_RESAMPLE_DET) ||
                   (x_out != x && y_out != y && (w == nullptr || w_out != w)),
               "resampling cannot run in place");
    PR_REQUIRE(ws_bytes >= hist_match_ws_bytes(n, k, grid->n_cells), "workspace too small: %zu < %zu", ws_bytes,
               hist_match_ws_bytes(n, k, grid->n_cells));
    const int I = grid->n_cells;
    HMatchArgs a{rho_t, rho_p, I, I, x, y, w, prior_stride, x_out, y_out, w_out, n, n, d, nullptr};
    return hist_match(kind, a, k, make_hgrid(grid), make_key(seed), instance, t_first, ws, as_stream(stream));
}

extern "C" int pr_parareal_hist_create(const pr_sde *sde, const pr_schedule *sched, const pr_grid *grid, uint64_t seed,
                                       uint32_t instance, int64_t n, int iterator, int matching, int flags,
                                       void *stream, void **h) {
    clear_error();
    PR_CHECK(check_sde(sde));
    PR_CHECK(check_schedule(sched));
    PR_CHECK(check_hist_grid(grid));
    PR_REQUIRE(h != nullptr, "h must be non-NULL");
    PR_REQUIRE(sde->precision == PR_F64, "histogram states run in FP64");
    PR_REQUIRE(iterator >= PR_J_ADD && iterator <= PR_J_QUANTILE, "unknown iterator %d", iterator);
    PR_REQUIRE(matching >= PR_M_MARGINAL && matching <= PR_M_RESAMPLE_DET, "unknown matching %d", matching);
    PR_REQUIRE(n >= 1 && n <= 0xFFFFFFFFll, "n must be in [1, 2^32)");
    PR_REQUIRE(sched->n_slices <= 1023, "at most 1023 slices");
    PR_REQUIRE((flags & ~(PR_REUSE_COARSE | PR_PROFILE)) == 0, "flags other than PR_REUSE_COARSE and PR_PROFILE");
    HistPR *p = nullptr;
    PR_CHECK(hist_parareal_create(sde, nullptr, sched, grid, seed, instance, n, iterator, matching, flags,
                                  as_stream(stream), &p));
    *h = p;
    return PR_OK;
}

extern "C" int pr_parareal_hist_create_chem(const pr_chem *c, const pr_schedule *sched, const pr_grid *grid,
                                            uint64_t seed, uint32_t instance, int64_t n, int iterator, int matching,
                                            int flags, void *stream, void **h) {
    clear_error();
    PR_CHECK(check_chem(c));
    PR_CHECK(check_schedule(sched));
    PR_CHECK(check_hist_grid(grid));
    PR_REQUIRE(h != nullptr, "h must be non-NULL");
    PR_REQUIRE(iterator >= PR_J_ADD && iterator <= PR_J_QUANTILE, "unknown iterator %d", iterator);
    PR_REQUIRE(matching >= PR_M_MARGINAL && matching <= PR_M_RESAMPLE_DET, "unknown matching %d", matching);
    PR_REQUIRE(n >= 1 && n <= 0xFFFFFFFFll, "n must be in [1, 2^32)");
    PR_REQUIRE(sched->n_slices <= 1023, "at most 1023 slices");
    PR_REQUIRE((flags & ~(PR_REUSE_COARSE | PR_PROFILE)) == 0, "flags other than PR_REUSE_COARSE and PR_PROFILE");
    HistPR *p = nullptr;
    PR_CHECK(hist_parareal_create(nullptr, c, sched, grid, seed, instance, n, iterator, matching, flags,
                                  as_stream(stream), &p));
    *h = p;
    return PR_OK;
}

extern "C" int pr_parareal_hist_iterate(void *h, int n_iter, const double *rho_ref, double *err_out, void *stream) {
    clear_error();
    PR_REQUIRE(h != nullptr && n_iter >= 0, "need a handle and n_iter >= 0");
    PR_REQUIRE(err_out == nullptr || rho_ref != nullptr, "err_out needs rho_ref");
    return hist_parareal_iterate((HistPR *)h, n_iter, rho_ref, err_out, as_stream(stream));
}

extern "C" int pr_parareal_hist_state(void *hv, int t, double *x, double *y, double *w, double *rho, void *stream) {
    clear_error();
    HistPR *h = (HistPR *)hv;
    PR_REQUIRE(h != nullptr, "NULL handle");
    PR_REQUIRE(t >= 0 && t <= h->K, "t must be in [0, %d]", h->K);
    hipStream_t st = as_stream(stream);
    const int64_t n = h->n;
    if (x) PR_CHECK(copy_d(x, h->xs(h->cur, t), sizeof(double) * n, st));
    if (y) PR_CHECK(copy_d(y, h->ys(h->cur, t), sizeof(double) * h->D * n, st));
    if (w) {
        if (h->weighted) {
            PR_CHECK(copy_d(w, h->wsl(h->cur, t), sizeof(double) * n, st));
        } else {
            hipLaunchKernelGGL(fill_f64, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0, st, w, n,
                               1.0 / (double)n);
            PR_LAUNCHED();
        }
    }
    if (rho) PR_CHECK(copy_d(rho, h->row(h->rho, t), sizeof(double) * h->I, st));
    return PR_OK;
}

extern "C" int pr_parareal_hist_iteration(const void *h) { return h ? ((const HistPR *)h)->k : -1; }

extern "C" int pr_parareal_hist_profile(const void *hv, double *ms_out, int *iterations) {
    clear_error();
    const HistPR *h = (const HistPR *)hv;
    PR_REQUIRE(h != nullptr && ms_out != nullptr, "need a handle and ms_out");
    PR_REQUIRE(h->flags & PR_PROFILE, "the handle was created without PR_PROFILE");
    for (int p = 0; p < PR_PH_COUNT; ++p) ms_out[p] = h->ph_ms[p];
    if (iterations) *iterations = h->timed;
    return PR_OK;
}

extern "C" int pr_parareal_hist_destroy(void *h) {
    clear_error();
    if (h) {
        (void)hipDeviceSynchronize();
        hist_free((HistPR *)h);
    }
    return PR_OK;
}

extern "C" int pr_parareal_fp_create(const void *fine, const void *coarse, const pr_grid *grid, const double *rho0,
                                     int iterator, int flags, void *stream, void **h) {
    clear_error();
    PR_CHECK(check_hist_grid(grid));
    PR_REQUIRE(fine != nullptr && coarse != nullptr && rho0 != nullptr && h != nullptr,
               "fine, coarse, rho0 and h must be non-NULL");
    PR_REQUIRE(iterator >= PR_J_ADD && iterator <= PR_J_QUANTILE, "unknown iterator %d", iterator);
    PR_REQUIRE(flags == 0, "no flags are defined for this driver");
    const Coarse *f = (const Coarse *)fine, *c = (const Coarse *)coarse;
    PR_REQUIRE(coarse_grid_cells(f) == grid->n_cells && coarse_grid_cells(c) == grid->n_cells,
               "both propagators must use the %d cells of the grid", grid->n_cells);
    PR_REQUIRE(coarse_n_slices(f) == coarse_n_slices(c), "fine and coarse propagators need the same slices");
    PR_REQUIRE(coarse_n_slices(c) <= 1023, "at most 1023 slices");
    FpPR *p = nullptr;
    PR_CHECK(fp_parareal_create(f, c, grid, rho0, iterator, as_stream(stream), &p));
    *h = p;
    return PR_OK;
}

extern "C" int pr_parareal_fp_iterate(void *h, int n_iter, const double *rho_ref, double *err_out, void *stream) {
    clear_error();
    PR_REQUIRE(h != nullptr && n_iter >= 0, "need a handle and n_iter >= 0");
    PR_REQUIRE(err_out == nullptr || rho_ref != nullptr, "err_out needs rho_ref");
    return fp_parareal_iterate((FpPR *)h, n_iter, rho_ref, err_out, as_stream(stream));
}

extern "C" int pr_parareal_fp_state(void *hv, int t, double *rho, void *stream) {
    clear_error();
    FpPR *h = (FpPR *)hv;
    PR_REQUIRE(h != nullptr && rho != nullptr, "need a handle and rho");
    PR_REQUIRE(t >= 0 && t <= h->K, "t must be in [0, %d]", h->K);
    return copy_d(rho, h->row(h->rho, t), sizeof(double) * h->I, as_stream(stream));
}

extern "C" int pr_parareal_fp_iteration(const void *h) { return h ? ((const FpPR *)h)->k : -1; }

extern "C" int pr_parareal_fp_destroy(void *h) {
    clear_error();
    if (h) {
        (void)hipDeviceSynchronize();
        fp_free((FpPR *)h);
    }
    return PR_OK;
}
