// Restriction to the empirical quantile function (Sec. 3.2.2, Sec. 4.4):
// a segmented, stable LSD radix sort of the slow coordinates of k ensembles
// (one segment per ensemble), followed by the midpoint (Hazen) knots; the
// moments (eq. (MCestimator)) and the cell histogram (eq. (binning)) are
// fused into the first read of the values.
//
// Sort design (HBM bound): 8-bit digits, one pass per byte of the orderable
// key.  A pass = count (digit histogram of each 4096-key tile) -> scan
// (per segment, digit-major over tiles, so equal digits keep tile order) ->
// scatter.  Inside a tile each wave ranks its 1024 keys in order with
// ballot-based peer masks, which keeps the pass stable; the tile is then
// staged in LDS in digit order so that each digit run is written to HBM as a
// contiguous burst.  The first pass reads the FP64 values directly and uses
// the particle index as payload; the last pass writes the outputs the caller
// asked for (rank by scatter, perm and sorted values in order).
#include "pr_internal.hpp"

namespace pr {

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_ITEMS = 16;
constexpr int RS_WAVE_KEYS = 64 * RS_ITEMS;      // 1024
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;   // 4096
constexpr int RS_RADIX = 256;

template <typename K> struct KeyTraits;
template <> struct KeyTraits<uint64_t> { using V = double; static constexpr int passes = 8; };
template <> struct KeyTraits<uint32_t> { using V = float;  static constexpr int passes = 4; };

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct HistArgs {
    uint32_t *hist;  // [k][cells] or NULL
    int cells;
    double lo, inv_h;
};

// ---------------------------------------------------------------------------
// Count: per-tile digit histogram.  Pass 0 also sums the four powers of x
// (fixed-order per tile) and fills the cell histogram.
// ---------------------------------------------------------------------------
template <typename K, bool FIRST>
__global__ void __launch_bounds__(RS_THREADS)
rs_count(const void *__restrict__ src, int shift, int64_t n, int nblk, uint32_t *__restrict__ counts,
         double *__restrict__ mom_part, HistArgs ha) {
    using V = typename KeyTraits<K>::V;
    __shared__ uint32_t h[RS_WAVES][RS_RADIX];
    __shared__ double wsum[RS_WAVES][4];
    extern __shared__ uint32_t cell_h[];
    const int seg = blockIdx.y, blk = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int i = tid; i < RS_WAVES * RS_RADIX; i += RS_THREADS) (&h[0][0])[i] = 0;
    const bool do_hist = FIRST && ha.hist != nullptr;
    if (do_hist)
        for (int i = tid; i < ha.cells; i += RS_THREADS) cell_h[i] = 0;
    __syncthreads();
    const int64_t seg_base = (int64_t)seg * n;
    const int64_t tile0 = (int64_t)blk * RS_TILE + wave * RS_WAVE_KEYS;
    double s1 = 0, s2 = 0, s3 = 0, s4 = 0;
#pragma unroll 4
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t idx = tile0 + i * 64 + lane;
        if (idx < n) {
            K key;
            if constexpr (FIRST) {
                const V v = ((const V *)src)[seg_base + idx];
                key = key_of(v);
                const double xv = (double)v;
                const double x2 = xv * xv;
                s1 += xv;
                s2 += x2;
                s3 += x2 * xv;
                s4 += x2 * x2;
                if (do_hist) {
                    double c = floor((xv - ha.lo) * ha.inv_h);
                    c = fmin(fmax(c, 0.0), (double)(ha.cells - 1));
                    atomicAdd(&cell_h[(int)c], 1u);
                }
            } else {
                key = ((const K *)src)[seg_base + idx];
            }
            atomicAdd(&h[wave][(uint32_t)(key >> shift) & 0xFFu], 1u);
        }
    }
    if (FIRST && mom_part != nullptr) {
        // fixed butterfly: every lane ends with the same total
        for (int off = 32; off >= 1; off >>= 1) {
            s1 += __shfl_xor(s1, off);
            s2 += __shfl_xor(s2, off);
            s3 += __shfl_xor(s3, off);
            s4 += __shfl_xor(s4, off);
        }
        if (lane == 0) {
            wsum[wave][0] = s1;
            wsum[wave][1] = s2;
            wsum[wave][2] = s3;
            wsum[wave][3] = s4;
        }
    }
    __syncthreads();
    {
        const int d = tid;  // RS_THREADS == RS_RADIX
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) c += h[w][d];
        counts[((int64_t)seg * RS_RADIX + d) * nblk + blk] = c;
    }
    if (FIRST && mom_part != nullptr && tid < 4) {
        double t = 0;
        for (int w = 0; w < RS_WAVES; ++w) t += wsum[w][tid];
        mom_part[((int64_t)seg * nblk + blk) * 4 + tid] = t;
    }
    if (do_hist)
        for (int i = tid; i < ha.cells; i += RS_THREADS)
            if (cell_h[i]) atomicAdd(&ha.hist[(int64_t)seg * ha.cells + i], cell_h[i]);
}

// ---------------------------------------------------------------------------
// Scan: exclusive prefix over the digit-major [256][nblk] counts of a segment.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) rs_scan(uint32_t *__restrict__ counts, int nblk) {
    __shared__ uint32_t wtot[16];
    const int seg = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t L = (int64_t)RS_RADIX * nblk;
    uint32_t *c = counts + (int64_t)seg * L;
    const int64_t chunk = (L + 1023) / 1024;
    const int64_t b = tid * chunk, e = (b + chunk < L) ? b + chunk : L;
    uint32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += c[i];
    // inclusive scan of s across the block
    uint32_t v = s;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    if (lane == 63) wtot[wave] = v;
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = 0;
        for (int w = 0; w < 16; ++w) {
            const uint32_t t = wtot[w];
            wtot[w] = acc;
            acc += t;
        }
    }
    __syncthreads();
    uint32_t run = v - s + wtot[wave];  // exclusive prefix of this thread's chunk
    for (int64_t i = b; i < e; ++i) {
        const uint32_t t = c[i];
        c[i] = run;
        run += t;
    }
}

// ---------------------------------------------------------------------------
// Scatter: stable rank inside the tile, LDS staging, contiguous writes.
// ---------------------------------------------------------------------------
template <typename K, bool FIRST, bool LAST>
__global__ void __launch_bounds__(RS_THREADS)
rs_scatter(const void *__restrict__ src, const uint32_t *__restrict__ vals_in, K *__restrict__ keys_out,
           uint32_t *__restrict__ vals_out, const uint32_t *__restrict__ offsets, int shift, int64_t n,
           int nblk, uint32_t *__restrict__ rank_out, uint32_t *__restrict__ perm_out,
           double *__restrict__ xs_out) {
    using V = typename KeyTraits<K>::V;
    __shared__ uint32_t wcnt[RS_WAVES][RS_RADIX];
    __shared__ uint32_t wbase[RS_WAVES][RS_RADIX];
    __shared__ uint32_t gdelta[RS_RADIX];
    __shared__ uint32_t wtot[RS_WAVES];
    __shared__ K skeys[RS_TILE];
    __shared__ uint32_t svals[RS_TILE];

    const int seg = blockIdx.y, blk = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t seg_base = (int64_t)seg * n;
    const int64_t tile0 = (int64_t)blk * RS_TILE + wave * RS_WAVE_KEYS;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    for (int i = lane; i < RS_RADIX; i += 64) wcnt[wave][i] = 0;
    wave_sync();

    K key[RS_ITEMS];
    uint32_t val[RS_ITEMS];
    uint32_t rnk[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t idx = tile0 + i * 64 + lane;
        if (idx < n) {
            if constexpr (FIRST) {
                key[i] = key_of(((const V *)src)[seg_base + idx]);
                val[i] = (uint32_t)idx;
            } else {
                key[i] = ((const K *)src)[seg_base + idx];
                val[i] = vals_in[seg_base + idx];
            }
        } else {
            key[i] = 0;
            val[i] = 0;
        }
    }
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const bool valid = tile0 + i * 64 + lane < n;
        const uint32_t d = (uint32_t)(key[i] >> shift) & 0xFFu;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        uint32_t base = 0;
        if (valid) base = wcnt[wave][d];
        rnk[i] = base + (uint32_t)__popcll(peers & lt);
        wave_sync();
        if (valid && lane == 63 - __clzll(peers)) wcnt[wave][d] = base + (uint32_t)__popcll(peers);
        wave_sync();
    }
    __syncthreads();
    {
        const int d = tid;
        uint32_t c[RS_WAVES], tot = 0;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) {
            c[w] = wcnt[w][d];
            tot += c[w];
        }
        // exclusive scan of tot over the 256 digits
        uint32_t v = tot;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t t = __shfl_up(v, off);
            if (lane >= off) v += t;
        }
        if (lane == 63) wtot[wave] = v;
        __syncthreads();
        uint32_t pre = 0;
        for (int w = 0; w < wave; ++w) pre += wtot[w];
        const uint32_t lstart = pre + v - tot;
        uint32_t acc = lstart;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) {
            wbase[w][d] = acc;
            acc += c[w];
        }
        gdelta[d] = offsets[((int64_t)seg * RS_RADIX + d) * nblk + blk] - lstart;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        if (tile0 + i * 64 + lane < n) {
            const uint32_t d = (uint32_t)(key[i] >> shift) & 0xFFu;
            const uint32_t lp = wbase[wave][d] + rnk[i];
            skeys[lp] = key[i];
            svals[lp] = val[i];
        }
    }
    __syncthreads();
    const int64_t rem = n - (int64_t)blk * RS_TILE;
    const int tile_n = rem < RS_TILE ? (int)rem : RS_TILE;
    for (int j = tid; j < tile_n; j += RS_THREADS) {
        const K k = skeys[j];
        const uint32_t v = svals[j];
        const uint32_t gpos = (uint32_t)j + gdelta[(uint32_t)(k >> shift) & 0xFFu];
        if ((int64_t)gpos >= n || (int64_t)v >= n) continue;  // unreachable for a consistent scan
        keys_out[seg_base + gpos] = k;
        if (!LAST || vals_out) vals_out[seg_base + gpos] = v;
        if (LAST) {
            if (rank_out) rank_out[seg_base + v] = gpos;
            if (perm_out) perm_out[seg_base + gpos] = v;
            if (xs_out) xs_out[seg_base + gpos] = value_of(k);
        }
    }
}

// ---------------------------------------------------------------------------
// Knots (midpoint convention) from the sorted keys; moment totals.
// ---------------------------------------------------------------------------
template <typename K>
__global__ void rs_knots(const K *__restrict__ sorted, int64_t n, int nq, double *__restrict__ q) {
#pragma clang fp contract(off)
    const int seg = blockIdx.x;
    const K *s = sorted + (int64_t)seg * n;
    for (int j = threadIdx.x; j <= nq; j += blockDim.x) {
        const double t = (double)((int64_t)j * n) / (double)nq - 0.5;
        double v;
        if (t <= 0.0) {
            v = value_of(s[0]);
        } else if (t >= (double)(n - 1)) {
            v = value_of(s[n - 1]);
        } else {
            const int64_t r = (int64_t)floor(t);
            const double f = t - (double)r;
            const double a = value_of(s[r]), b = value_of(s[r + 1]);
            v = a + f * (b - a);
            v = v < b ? v : b;
        }
        q[(int64_t)seg * (nq + 1) + j] = v;
    }
}

__global__ void rs_moments(const double *__restrict__ part, int nblk, int64_t n, double *__restrict__ mom) {
    const int seg = blockIdx.x, lane = threadIdx.x;  // one wave
    for (int m = 0; m < 4; ++m) {
        double s = 0;
        for (int b = lane; b < nblk; b += 64) s += part[((int64_t)seg * nblk + b) * 4 + m];
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) mom[seg * 4 + m] = s / (double)n;
    }
}

__global__ void zero_u32(uint32_t *p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static int rs_nblk(int64_t n) { return (int)((n + RS_TILE - 1) / RS_TILE); }

size_t restrict_ws(int64_t n, int k, int precision) {
    const size_t ks = precision == PR_F32 ? 4 : 8;
    const size_t nk = (size_t)n * (size_t)k;
    const size_t nb = (size_t)rs_nblk(n);
    return align256(nk * ks) * 2 + align256(nk * 4) * 2 + align256(nb * RS_RADIX * k * 4) +
           align256(nb * k * 4 * 8) + 256;
}

template <typename K>
static int restrict_impl(const void *x, int64_t n, int k, int nq, const pr_grid *hg, double *q,
                         uint32_t *rank, uint32_t *perm, double *xs, double *mom, uint32_t *hist,
                         void *ws, hipStream_t st) {
    const int nblk = rs_nblk(n);
    const size_t nk = (size_t)n * (size_t)k;
    char *p = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    K *keys[2];
    uint32_t *vals[2];
    keys[0] = (K *)p; p += align256(nk * sizeof(K));
    keys[1] = (K *)p; p += align256(nk * sizeof(K));
    vals[0] = (uint32_t *)p; p += align256(nk * 4);
    vals[1] = (uint32_t *)p; p += align256(nk * 4);
    uint32_t *counts = (uint32_t *)p; p += align256((size_t)nblk * RS_RADIX * k * 4);
    double *mom_part = (double *)p;

    HistArgs ha{hist, 0, 0.0, 0.0};
    size_t cell_lds = 0;
    if (hist) {
        ha.cells = hg->n_cells;
        ha.lo = hg->x_lo;
        ha.inv_h = (double)hg->n_cells / (hg->x_hi - hg->x_lo);
        cell_lds = (size_t)hg->n_cells * 4;
        const int64_t cnt = (int64_t)k * hg->n_cells;
        hipLaunchKernelGGL(zero_u32, dim3((unsigned)((cnt + 255) / 256 < 1024 ? (cnt + 255) / 256 : 1024)),
                           dim3(256), 0, st, hist, cnt);
        PR_LAUNCHED();
    }
    constexpr int P = KeyTraits<K>::passes;
    const dim3 grid(nblk, k);
    for (int pass = 0; pass < P; ++pass) {
        const int shift = 8 * pass;
        const int in = (pass + 1) & 1, out = pass & 1;  // pass 0 writes buffer 0
        if (pass == 0) {
            hipLaunchKernelGGL((rs_count<K, true>), grid, dim3(RS_THREADS), cell_lds, st, x, shift, n, nblk,
                               counts, mom ? mom_part : nullptr, ha);
        } else {
            hipLaunchKernelGGL((rs_count<K, false>), grid, dim3(RS_THREADS), 0, st, (const void *)keys[in],
                               shift, n, nblk, counts, nullptr, HistArgs{nullptr, 0, 0.0, 0.0});
        }
        PR_LAUNCHED();
        hipLaunchKernelGGL(rs_scan, dim3(k), dim3(1024), 0, st, counts, nblk);
        PR_LAUNCHED();
        const bool last = pass == P - 1;
        if (pass == 0) {
            hipLaunchKernelGGL((rs_scatter<K, true, false>), grid, dim3(RS_THREADS), 0, st, x, nullptr,
                               keys[out], vals[out], counts, shift, n, nblk, nullptr, nullptr, nullptr);
        } else if (!last) {
            hipLaunchKernelGGL((rs_scatter<K, false, false>), grid, dim3(RS_THREADS), 0, st,
                               (const void *)keys[in], vals[in], keys[out], vals[out], counts, shift, n, nblk,
                               nullptr, nullptr, nullptr);
        } else {
            hipLaunchKernelGGL((rs_scatter<K, false, true>), grid, dim3(RS_THREADS), 0, st,
                               (const void *)keys[in], vals[in], keys[out], (uint32_t *)nullptr, counts, shift,
                               n, nblk, rank, perm, xs);
        }
        PR_LAUNCHED();
    }
    const K *sorted = keys[(P - 1) & 1];
    hipLaunchKernelGGL((rs_knots<K>), dim3(k), dim3(128), 0, st, sorted, n, nq, q);
    PR_LAUNCHED();
    if (mom) {
        hipLaunchKernelGGL(rs_moments, dim3(k), dim3(64), 0, st, mom_part, nblk, n, mom);
        PR_LAUNCHED();
    }
    return PR_OK;
}

int restrict_quantiles(const void *x, int precision, int64_t n, int k, int nq, const pr_grid *hg, double *q,
                       uint32_t *rank, uint32_t *perm, double *xs, double *mom, uint32_t *hist, void *ws,
                       hipStream_t st) {
    if (precision == PR_F64)
        return restrict_impl<uint64_t>(x, n, k, nq, hg, q, rank, perm, xs, mom, hist, ws, st);
    return restrict_impl<uint32_t>(x, n, k, nq, hg, q, rank, perm, xs, mom, hist, ws, st);
}

}  // namespace pr

using namespace pr;

extern "C" size_t pr_restrict_workspace_size(int64_t n, int k, int precision) {
    if (n <= 0 || k <= 0) return 256;
    return restrict_ws(n, k, precision);
}

extern "C" int pr_restrict_quantiles(const void *x, int precision, int64_t n, int k, int n_q,
                                     const pr_grid *hist_grid, double *q, uint32_t *rank, uint32_t *perm,
                                     double *x_sorted, double *moments, uint32_t *hist, void *ws,
                                     size_t ws_bytes, void *stream) {
    clear_error();
    PR_REQUIRE(valid_precision(precision), "precision must be 64 or 32");
    PR_REQUIRE(n >= 1 && n <= 0xFFFFFFFFll, "n must be in [1, 2^32)");
    PR_REQUIRE(k >= 1 && k <= 65535, "k must be in [1, 65535]");
    PR_REQUIRE(n_q >= 1 && n_q <= 1 << 20, "n_q must be in [1, 2^20]");
    PR_REQUIRE(x != nullptr && q != nullptr && ws != nullptr, "x, q and ws must be non-NULL");
    PR_REQUIRE((int64_t)n * k <= 0x7FFFFFFFFFFFll, "n * k too large");
    if (hist) {
        PR_REQUIRE(hist_grid != nullptr, "hist requires hist_grid");
        PR_REQUIRE(hist_grid->n_cells >= 1 && hist_grid->n_cells <= 8192 && hist_grid->x_lo < hist_grid->x_hi,
                   "hist_grid must have 1..8192 cells and x_lo < x_hi");
    }
    if (ws_bytes < restrict_ws(n, k, precision)) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, restrict_ws(n, k, precision));
        return PR_E_NOMEM;
    }
    return restrict_quantiles(x, precision, n, k, n_q, hist_grid, q, rank, perm, x_sorted, moments, hist, ws,
                              as_stream(stream));
}
