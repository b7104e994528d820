// Restriction to the empirical quantile function (Sec. 3.2.2, Sec. 4.4):
// a segmented sort of the slow coordinates of many ensembles (one segment
// per ensemble, equal or unequal lengths) by (key, particle), followed by
// the midpoint (Hazen) knots; the moments (eq. (MCestimator)) and the cell
// histogram (eq. (binning)) are fused into the first read of the values.
// FP64 ensembles of SS_MIN_N..SS_MAX_N keys with ranks or the permutation
// asked for take the splitter sort (sample, buckets, one LDS sort per
// bucket; described with its kernels below); the rest take the radix sort.
//
// Radix sort design (HBM bound): 8-bit digits, one pass per byte of the
// orderable key.  A pass is
//   count   digit histogram of every tile (ITEMS x 256 keys),
//   rowscan one wave per (segment, digit) -- one block per segment in the
//           segment-table layout: exclusive prefix of that digit's tile
//           counts and the digit total of the segment,
//   scatter stable rank of every key inside its tile (each wave ranks its
//           keys in order with ballot-built peer masks), exclusive scan of
//           the digit totals, then the tile is staged in LDS in digit order
//           and every digit run is written to HBM as a contiguous burst.
// Equal digits keep tile order, so every pass is stable and the sort orders
// by (key, particle).  The first pass reads FP64 (or FP32) values directly
// and generates the particle index as payload; the last pass writes the
// outputs asked for (rank by scatter, perm and sorted values in order).  A
// sort that only needs knots carries no payload.  64-bit keys run only the
// four passes over their high halves, then a fix-up pass (rs_fixup) that
// orders every run of equal high halves and writes the last pass's outputs
// (the ranks through a staging buffer instead of stores to random addresses,
// rs_rank_bucket and rs_rank_place); the complete sort follows, guarded by a
// flag that the fix-up raises only for a run longer than it handles.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "pr_internal.hpp"

namespace pr {

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_RADIX = 256;
constexpr int RS_ITEMS = 16;  // keys per thread and tile (tiles of RS_THREADS x RS_ITEMS keys)

template <typename K> struct KeyTraits;
template <> struct KeyTraits<uint64_t> { using V = double; static constexpr int passes = 8; };
template <> struct KeyTraits<uint32_t> { using V = float;  static constexpr int passes = 4; };

// Key buffer (0 or 1) of the workspace that holds the sorted keys when a
// sort ends: 64-bit keys end in buffer 0 (the fix-up after the passes over
// the high halves, or the complete sort arranged to end there), 32-bit keys
// in the buffer the last of their 4 passes writes.
template <typename K>
constexpr int sorted_buffer() { return std::is_same<K, uint64_t>::value ? 0 : 1; }

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive prefix of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_exclusive_256(uint32_t v, uint32_t *wtot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(inc, off);
        if (lane >= off) inc += t;
    }
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wave; ++w) pre += wtot[w];
    __syncthreads();
    return pre + inc - v;
}

struct HistArgs {
    uint32_t *hist;  // [segments][cells] or NULL
    int cells;
    double lo, inv_h;
};

struct TileRef {
    int seg, blk, nblk;
    int64_t base, n, tile0;
};

// Tile processed by block b of nb.  Blocks are handed to the 8 XCDs round
// robin (block b runs on XCD b mod 8) and every XCD has its own L2, so each
// XCD takes one contiguous range of tiles: neighbouring tiles share cache
// lines of the per-tile count columns and of the digit runs they write, and
// those lines then fill up in one L2 instead of being written partially from
// several.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
    constexpr int64_t X = 8;
    const int64_t q = nb / X, r = nb % X;
    const int64_t x = b % X, i = b / X;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

template <bool VAR>
__device__ __forceinline__ TileRef tile_ref(const SortLayout &L, int64_t t) {
    TileRef r;
    if constexpr (VAR) {
        r.seg = L.tile_seg[t];
        const SortSeg s = L.segs[r.seg];
        r.blk = (int)(t - s.tile0);
        r.nblk = s.nblk;
        r.base = s.base;
        r.n = s.n;
        r.tile0 = s.tile0;
    } else {
        r.seg = (int)(t / L.nblk);
        r.blk = (int)(t % L.nblk);
        r.nblk = L.nblk;
        r.base = (int64_t)r.seg * L.n;
        r.n = L.n;
        r.tile0 = (int64_t)r.seg * L.nblk;
    }
    return r;
}

template <bool VAR>
__device__ __forceinline__ void seg_ref(const SortLayout &L, int s, int64_t &base, int64_t &n, int64_t &tile0,
                                        int &nblk, int &qrow) {
    if constexpr (VAR) {
        const SortSeg g = L.segs[s];
        base = g.base;
        n = g.n;
        tile0 = g.tile0;
        nblk = g.nblk;
        qrow = g.qrow;
    } else {
        base = (int64_t)s * L.n;
        n = L.n;
        tile0 = (int64_t)s * L.nblk;
        nblk = L.nblk;
        qrow = s;
    }
}

// ---------------------------------------------------------------------------
// Count.
// ---------------------------------------------------------------------------
template <typename K, int ITEMS, bool FIRST, bool VAR>
__global__ void __launch_bounds__(RS_THREADS)
rs_count(const void *__restrict__ src, int shift, SortLayout L, uint32_t *__restrict__ counts,
         double *__restrict__ mom_part, HistArgs ha) {
    using V = typename KeyTraits<K>::V;
    constexpr int WAVE_KEYS = 64 * ITEMS, TILE = RS_THREADS * ITEMS;
    // two copies of every wave's histogram (even and odd lanes) halve the
    // same-address serialisation of the LDS atomics when few digits occur
    __shared__ uint32_t h[RS_WAVES][2][RS_RADIX];
    __shared__ double wsum[RS_WAVES][4];
    extern __shared__ uint32_t cell_h[];
    if (L.guard && *L.guard == 0) return;
    const TileRef T = tile_ref<VAR>(L, xcd_tile(blockIdx.x, gridDim.x));
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int i = tid; i < RS_WAVES * 2 * RS_RADIX; i += RS_THREADS) (&h[0][0][0])[i] = 0;
    const bool do_hist = FIRST && ha.hist != nullptr;
    if (do_hist)
        for (int i = tid; i < ha.cells; i += RS_THREADS) cell_h[i] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)T.blk * TILE + wave * WAVE_KEYS;
    // all loads of the tile first, so that they are in flight together
    using In = typename std::conditional<FIRST, V, K>::type;
    In in[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = t0 + i * 64 + lane;
        in[i] = idx < T.n ? ((const In *)src)[T.base + idx] : (In)0;
    }
    double s1 = 0, s2 = 0, s3 = 0, s4 = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = t0 + i * 64 + lane;
        if (idx < T.n) {
            K key;
            if constexpr (FIRST) {
                const V v = in[i];
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
                key = in[i];
            }
            atomicAdd(&h[wave][lane & 1][(uint32_t)(key >> shift) & 0xFFu], 1u);
        }
    }
    if (FIRST && mom_part != nullptr) {
        for (int off = 32; off >= 1; off >>= 1) {  // fixed butterfly
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
        for (int w = 0; w < RS_WAVES; ++w) c += h[w][0][d] + h[w][1][d];
        counts[T.tile0 * RS_RADIX + (int64_t)d * T.nblk + T.blk] = c;
    }
    if (FIRST && mom_part != nullptr && tid < 4) {
        double t = 0;
        for (int w = 0; w < RS_WAVES; ++w) t += wsum[w][tid];
        mom_part[(T.tile0 + T.blk) * 4 + tid] = t;
    }
    if (do_hist)
        for (int i = tid; i < ha.cells; i += RS_THREADS)
            if (cell_h[i]) atomicAdd(&ha.hist[(int64_t)T.seg * ha.cells + i], cell_h[i]);
}

// ---------------------------------------------------------------------------
// Row scan: one wave per (segment, digit).
// ---------------------------------------------------------------------------
template <bool VAR>
__global__ void __launch_bounds__(256) rs_rowscan(uint32_t *__restrict__ counts, uint32_t *__restrict__ totals,
                                                  SortLayout L) {
    if (L.guard && *L.guard == 0) return;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= (int64_t)L.nseg * RS_RADIX) return;
    const int lane = threadIdx.x & 63;
    const int s = (int)(row >> 8), d = (int)(row & 255);
    int64_t base, n, tile0;
    int nblk, qrow;
    seg_ref<VAR>(L, s, base, n, tile0, nblk, qrow);
    uint32_t *c = counts + tile0 * RS_RADIX + (int64_t)d * nblk;
    uint32_t carry = 0;
    for (int c0 = 0; c0 < nblk; c0 += 64) {
        const int i = c0 + lane;
        const uint32_t v = i < nblk ? c[i] : 0u;
        uint32_t inc = v;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t t = __shfl_up(inc, off);
            if (lane >= off) inc += t;
        }
        if (i < nblk) c[i] = carry + inc - v;
        carry += __shfl(inc, 63);
    }
    if (lane == 0) totals[(int64_t)s * RS_RADIX + d] = carry;
}

// Row scan for many short segments (the segment-table layout): one block per
// segment, one thread per digit walking that digit's tile counts, so that a
// launch has one block per segment instead of one wave per (segment, digit).
template <bool VAR>
__global__ void __launch_bounds__(256) rs_rowscan_seg(uint32_t *__restrict__ counts, uint32_t *__restrict__ totals,
                                                      SortLayout L) {
    if (L.guard && *L.guard == 0) return;
    const int s = blockIdx.x, d = threadIdx.x;  // RS_RADIX threads
    int64_t base, n, tile0;
    int nblk, qrow;
    seg_ref<VAR>(L, s, base, n, tile0, nblk, qrow);
    uint32_t *c = counts + tile0 * RS_RADIX + (int64_t)d * nblk;
    uint32_t carry = 0;
    for (int b = 0; b < nblk; ++b) {
        const uint32_t v = c[b];
        c[b] = carry;
        carry += v;
    }
    totals[(int64_t)s * RS_RADIX + d] = carry;
}

// ---------------------------------------------------------------------------
// Scatter.
// ---------------------------------------------------------------------------
template <typename K, int ITEMS, bool FIRST, bool LAST, bool PAYLOAD, bool VAR>
__global__ void __launch_bounds__(RS_THREADS)
rs_scatter(const void *__restrict__ src, const uint32_t *__restrict__ vals_in, K *__restrict__ keys_out,
           uint32_t *__restrict__ vals_out, const uint32_t *__restrict__ counts,
           const uint32_t *__restrict__ totals, int shift, SortLayout L, uint32_t *__restrict__ rank_out,
           uint32_t *__restrict__ perm_out, double *__restrict__ xs_out) {
    using V = typename KeyTraits<K>::V;
    constexpr int WAVE_KEYS = 64 * ITEMS, TILE = RS_THREADS * ITEMS;
    __shared__ uint32_t wcnt[RS_WAVES][RS_RADIX];
    __shared__ uint32_t wbase[RS_WAVES][RS_RADIX];
    __shared__ uint32_t gdelta[RS_RADIX];
    __shared__ uint32_t wtot[RS_WAVES];
    __shared__ K stage[TILE];  // keys, then (reused) payload

    if (L.guard && *L.guard == 0) return;
    const TileRef T = tile_ref<VAR>(L, xcd_tile(blockIdx.x, gridDim.x));
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t t0 = (int64_t)T.blk * TILE + wave * WAVE_KEYS;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    for (int i = lane; i < RS_RADIX; i += 64) wcnt[wave][i] = 0;
    wave_sync();

    K key[ITEMS];
    uint32_t val[ITEMS];
    uint32_t rnk[ITEMS];
    // all loads of the tile first, so that they are in flight together (a
    // conversion next to each load made every load wait for the one before)
    using In = typename std::conditional<FIRST, V, K>::type;
    In in[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = t0 + i * 64 + lane;
        in[i] = idx < T.n ? ((const In *)src)[T.base + idx] : (In)0;
        val[i] = 0;
        if constexpr (PAYLOAD && !FIRST)
            if (idx < T.n) val[i] = vals_in[T.base + idx];
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = t0 + i * 64 + lane;
        key[i] = 0;
        if (idx < T.n) {
            if constexpr (FIRST) {
                key[i] = key_of(in[i]);
                val[i] = (uint32_t)idx;
            } else {
                key[i] = in[i];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const bool valid = t0 + i * 64 + lane < T.n;
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
        const uint32_t lstart = block_exclusive_256(tot, wtot);
        const uint32_t dbase = block_exclusive_256(totals[(int64_t)T.seg * RS_RADIX + d], wtot);
        uint32_t acc = lstart;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) {
            wbase[w][d] = acc;
            acc += c[w];
        }
        gdelta[d] = dbase + counts[T.tile0 * RS_RADIX + (int64_t)d * T.nblk + T.blk] - lstart;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (t0 + i * 64 + lane < T.n) {
            const uint32_t d = (uint32_t)(key[i] >> shift) & 0xFFu;
            stage[wbase[wave][d] + rnk[i]] = key[i];
        }
    }
    __syncthreads();
    const int64_t rem = T.n - (int64_t)T.blk * TILE;
    const int tile_n = rem < TILE ? (int)rem : TILE;
    uint32_t gpos[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int j = tid + r * RS_THREADS;
        gpos[r] = 0xFFFFFFFFu;
        if (j < tile_n) {
            const K k = stage[j];
            const uint32_t g = (uint32_t)j + gdelta[(uint32_t)(k >> shift) & 0xFFu];
            if ((int64_t)g < T.n) {  // always true for a consistent scan
                gpos[r] = g;
                keys_out[T.base + g] = k;
                if (LAST && xs_out) xs_out[T.base + g] = value_of(k);
            }
        }
    }
    if constexpr (PAYLOAD) {
        __syncthreads();
        uint32_t *sv = (uint32_t *)stage;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (t0 + i * 64 + lane < T.n) {
                const uint32_t d = (uint32_t)(key[i] >> shift) & 0xFFu;
                sv[wbase[wave][d] + rnk[i]] = val[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const int j = tid + r * RS_THREADS;
            if (j < tile_n && gpos[r] != 0xFFFFFFFFu) {
                const uint32_t v = sv[j];
                if (!LAST) {
                    vals_out[T.base + gpos[r]] = v;
                } else if ((int64_t)v < T.n) {
                    if (rank_out) rank_out[T.base + v] = gpos[r];
                    if (perm_out) perm_out[T.base + gpos[r]] = v;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Splitter sort of large FP64 ensembles (SS_MIN_N <= n <= SS_MAX_N; equal
// lengths or a segment table): the keys of every ensemble are first
// distributed over ss_buckets(n) buckets (about 4096 keys each) by splitters
// drawn from a sample, then every bucket is ordered on its own in LDS.
//   ss_sample_runs  SS_RUNS blocks per ensemble, each sorting SS_RUN keys of
//                   the sample (positions i n / (SS_RUNS SS_RUN)) in LDS and
//                   keeping its SS_B quantile keys;
//   ss_splitters    splitter b = the mean over the runs of their quantile
//                   value at level b / ss_buckets(n) (non-decreasing in b,
//                   as every run's quantiles are);
//   ss_count        bucket histogram of every tile and the bucket of every
//                   key (one byte; the moments and the cell histogram fused
//                   into this first read of the values);
//   rs_rowscan(_seg) tile offsets and bucket totals, as for a radix pass;
//   ss_scatter      scatter of (key, particle) into the buckets (in any
//                   order inside a bucket: slots from LDS atomics);
//   ss_bucket_sort  one block per bucket: the keys go to value sub-buckets
//                   (linear in the value between the bucket's bounds, which
//                   keeps the order), every key counts the keys of its
//                   sub-bucket that precede it by (key, particle), the
//                   particles read only for equal keys, and the bucket is
//                   written out in order with its permutation.
// A bucket above SS_CAP keys or a sub-bucket above SS_SUBMAX raises the flag
// that runs the complete radix sort behind it.  Compared with four radix
// passes and the fix-up this moves about half the bytes per key.
// ---------------------------------------------------------------------------
constexpr int SS_B = 256;
constexpr int SS_RUNS = 16;
constexpr int SS_RUN = 1024;
constexpr int SS_BT = 1024;                 // threads of a bucket block
constexpr int SS_IT = 7;                    // keys per thread of a bucket block
constexpr int SS_CAP = SS_BT * SS_IT;       // 7168: two bucket blocks share a CU's LDS
constexpr int SS_SUB = 2048;
constexpr int SS_SUBMAX = 512;
constexpr int64_t SS_MIN_N = (int64_t)1 << 16;
// Above this the SS_B buckets average more than 4352 keys, and the largest of
// them (about 1.5 times the mean with 64 samples per bucket) nears SS_CAP.
constexpr int64_t SS_MAX_N = ((int64_t)1 << 20) + ((int64_t)1 << 16);
static_assert(SS_B == RS_RADIX, "buckets take the place of a radix pass's digits");

// Buckets of an ensemble of n keys: about 4096 keys each, between 1 and SS_B.
__host__ __device__ __forceinline__ int ss_buckets(int64_t n) {
    const int64_t b = n >> 12;
    return b < 1 ? 1 : (b > SS_B ? SS_B : (int)b);
}
static_assert(SS_SUB == 2 * SS_BT, "two sub-bucket counts per thread");

// Bucket of a key: the number of splitters sp[1..SS_B-1] at or below it.
__device__ __forceinline__ uint32_t ss_bucket_of(uint64_t key, const uint64_t *sp) {
    uint32_t b = 0;
#pragma unroll
    for (uint32_t step = SS_B / 2; step >= 1; step >>= 1)
        if (sp[b + step] <= key) b += step;
    return b;
}

template <bool VAR>
__global__ void __launch_bounds__(SS_RUN / 2) ss_sample_runs(const double *__restrict__ x, SortLayout L,
                                                            uint64_t *__restrict__ runq) {
    __shared__ uint64_t sk[SS_RUN];
    const int r = blockIdx.x, s = blockIdx.y, t = threadIdx.x;
    int64_t base, n, tile0;
    int nblk, qrow;
    seg_ref<VAR>(L, s, base, n, tile0, nblk, qrow);
    const int64_t total = (int64_t)SS_RUNS * SS_RUN;
    const double *xs = x + base;
    for (int i = t; i < SS_RUN; i += blockDim.x) {
        const int64_t g = (int64_t)r * SS_RUN + i;
        sk[i] = key_of(xs[g * n / total]);
    }
    __syncthreads();
    for (int size = 2; size <= SS_RUN; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int lo = 2 * t - (t & (stride - 1)), hi = lo + stride;  // one pair per thread
            const bool up = (lo & size) == 0;
            const uint64_t a = sk[lo], b = sk[hi];
            if ((a > b) == up) {
                sk[lo] = b;
                sk[hi] = a;
            }
            __syncthreads();
        }
    for (int b = t; b < SS_B; b += blockDim.x)
        runq[((int64_t)s * SS_RUNS + r) * SS_B + b] = sk[b * (SS_RUN / SS_B)];
}

// Splitter b of an ensemble with B buckets: the mean over the runs of their
// quantile value at level b/B (the run's quantile b SS_B / B), each value
// first clamped to the finite range (infinities and NaN to the end of the
// range their key sorts to).  The clamped value is non-decreasing in the
// key, so the means are non-decreasing in b; averaging in the value domain
// keeps the splitters where the values lie (the key domain is far from
// linear in the value around 0).  Splitters B..SS_B-1 are the largest key:
// buckets past B stay empty (a key equal to it goes to bucket B - 1).
template <bool VAR>
__global__ void __launch_bounds__(SS_B) ss_splitters(const uint64_t *__restrict__ runq, SortLayout L,
                                                     uint64_t *__restrict__ split) {
#pragma clang fp contract(off)
    const int s = blockIdx.x, b = threadIdx.x;
    int64_t base, n, tile0;
    int nblk, qrow;
    seg_ref<VAR>(L, s, base, n, tile0, nblk, qrow);
    const int nb = ss_buckets(n);
    if (b >= nb) {
        split[(int64_t)s * SS_B + b] = ~0ull;
        return;
    }
    const int j = (int)(((int64_t)b * SS_B) / nb);
    double acc = 0.0;
    for (int r = 0; r < SS_RUNS; ++r) {
        const uint64_t k = runq[((int64_t)s * SS_RUNS + r) * SS_B + j];
        double v = value_of(k);
        if (v != v) v = (k >> 63) ? 1.79e308 : -1.79e308;
        v = fmin(fmax(v, -1.79e308), 1.79e308);
        acc += v / (double)SS_RUNS;
    }
    split[(int64_t)s * SS_B + b] = b == 0 ? 0ull : key_of(acc);
}

// The tiles of the radix passes (RS_THREADS x RS_ITEMS keys) are taken by
// twice the threads with half the keys each in the splitter sort's
// per-key passes.
constexpr int SC_THREADS = 2 * RS_THREADS;
constexpr int SC_WAVES = SC_THREADS / 64;

template <bool VAR>
__global__ void __launch_bounds__(SC_THREADS)
ss_count(const double *__restrict__ src, const uint64_t *__restrict__ split, SortLayout L,
         uint32_t *__restrict__ counts, double *__restrict__ mom_part, HistArgs ha, uint8_t *__restrict__ bucket) {
    constexpr int TILE = RS_THREADS * RS_ITEMS, ITEMS = TILE / SC_THREADS, WAVE_KEYS = 64 * ITEMS;
    __shared__ uint32_t h[SC_WAVES][2][RS_RADIX];
    __shared__ double wsum[SC_WAVES][4];
    __shared__ uint64_t sp[SS_B];
    extern __shared__ uint32_t cell_h[];
    const TileRef T = tile_ref<VAR>(L, xcd_tile(blockIdx.x, gridDim.x));
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int i = tid; i < SC_WAVES * 2 * RS_RADIX; i += SC_THREADS) (&h[0][0][0])[i] = 0;
    for (int i = tid; i < SS_B; i += SC_THREADS) sp[i] = split[(int64_t)T.seg * SS_B + i];
    const bool do_hist = ha.hist != nullptr;
    if (do_hist)
        for (int i = tid; i < ha.cells; i += SC_THREADS) cell_h[i] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)T.blk * TILE + wave * WAVE_KEYS;
    double in[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = t0 + i * 64 + lane;
        in[i] = idx < T.n ? src[T.base + idx] : 0.0;
    }
    // every key's bucket first (loads of LDS only, so the searches of the
    // tile's keys overlap), then the counting
    uint32_t bk[ITEMS];
    const uint32_t last = (uint32_t)ss_buckets(T.n) - 1;  // the largest key joins the last bucket
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t b = ss_bucket_of(key_of(in[i]), sp);
        bk[i] = b < last ? b : last;
    }
    // every key's bucket for the scatter, one byte each
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = t0 + i * 64 + lane;
        if (idx < T.n) bucket[T.base + idx] = (uint8_t)bk[i];
    }
    double s1 = 0, s2 = 0, s3 = 0, s4 = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = t0 + i * 64 + lane;
        if (idx < T.n) {
            const double xv = in[i];
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
            atomicAdd(&h[wave][lane & 1][bk[i]], 1u);
        }
    }
    if (mom_part != nullptr) {
        for (int off = 32; off >= 1; off >>= 1) {  // fixed butterfly, as in rs_count
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
    if (tid < RS_RADIX) {
        const int d = tid;
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < SC_WAVES; ++w) c += h[w][0][d] + h[w][1][d];
        counts[T.tile0 * RS_RADIX + (int64_t)d * T.nblk + T.blk] = c;
    }
    if (mom_part != nullptr && tid < 4) {
        double t = 0;
        for (int w = 0; w < SC_WAVES; ++w) t += wsum[w][tid];
        mom_part[(T.tile0 + T.blk) * 4 + tid] = t;
    }
    if (do_hist)
        for (int i = tid; i < ha.cells; i += SC_THREADS)
            if (cell_h[i]) atomicAdd(&ha.hist[(int64_t)T.seg * ha.cells + i], cell_h[i]);
}

// Exclusive prefix of one value per thread over a block of NT threads.
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t *wtot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(inc, off);
        if (lane >= off) inc += t;
    }
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wave; ++w) pre += wtot[w];
    __syncthreads();
    return pre + inc - v;
}

// Scatter of (key, particle) into the buckets.  The order inside a bucket
// is left to the block's LDS atomics: the bucket sort orders by (key,
// particle) whatever order its input has.
template <bool VAR>
__global__ void __launch_bounds__(SC_THREADS)
ss_scatter(const double *__restrict__ src, const uint8_t *__restrict__ bucket, uint64_t *__restrict__ keys_out,
           uint32_t *__restrict__ vals_out, const uint32_t *__restrict__ counts,
           const uint32_t *__restrict__ totals, SortLayout L, uint32_t *__restrict__ bstart) {
    constexpr int TILE = RS_THREADS * RS_ITEMS, ITEMS = TILE / SC_THREADS, WAVE_KEYS = 64 * ITEMS;
    __shared__ uint32_t bcnt[RS_RADIX];
    __shared__ uint32_t lstart[RS_RADIX];
    __shared__ uint32_t gdelta[RS_RADIX];
    __shared__ uint32_t wtot[SC_THREADS / 64];
    __shared__ uint64_t stage[TILE];
    __shared__ uint8_t sdig[TILE];

    const TileRef T = tile_ref<VAR>(L, xcd_tile(blockIdx.x, gridDim.x));
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t t0 = (int64_t)T.blk * TILE + wave * WAVE_KEYS;
    if (tid < RS_RADIX) bcnt[tid] = 0;
    __syncthreads();

    // bucket (low byte) and slot among the tile's keys of that bucket
    uint32_t dr[ITEMS];
    double in[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = t0 + i * 64 + lane;
        in[i] = idx < T.n ? src[T.base + idx] : 0.0;
        dr[i] = idx < T.n ? (uint32_t)bucket[T.base + idx] : 0u;
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if (t0 + i * 64 + lane < T.n) dr[i] |= atomicAdd(&bcnt[dr[i]], 1u) << 8;
    __syncthreads();
    {
        // one thread per bucket; the other half adds zeros to the scans
        const int d = tid & (RS_RADIX - 1);
        const bool own = tid < RS_RADIX;
        const uint32_t ls = block_exclusive<SC_THREADS>(own ? bcnt[d] : 0u, wtot);
        const uint32_t dbase = block_exclusive<SC_THREADS>(own ? totals[(int64_t)T.seg * RS_RADIX + d] : 0u, wtot);
        if (own) {
            lstart[d] = ls;
            gdelta[d] = dbase + counts[T.tile0 * RS_RADIX + (int64_t)d * T.nblk + T.blk] - ls;
            if (T.blk == 0) bstart[(int64_t)T.seg * RS_RADIX + d] = dbase;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if (t0 + i * 64 + lane < T.n) {
            const uint32_t j = lstart[dr[i] & 0xFFu] + (dr[i] >> 8);
            stage[j] = key_of(in[i]);
            sdig[j] = (uint8_t)dr[i];
        }
    __syncthreads();
    const int64_t rem = T.n - (int64_t)T.blk * TILE;
    const int tile_n = rem < TILE ? (int)rem : TILE;
    uint32_t gpos[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int j = tid + r * SC_THREADS;
        gpos[r] = 0xFFFFFFFFu;
        if (j < tile_n) {
            const uint32_t g = (uint32_t)j + gdelta[sdig[j]];
            if ((int64_t)g < T.n) {  // always true for a consistent scan
                gpos[r] = g;
                keys_out[T.base + g] = stage[j];
            }
        }
    }
    __syncthreads();
    uint32_t *sv = (uint32_t *)stage;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if (t0 + i * 64 + lane < T.n) sv[lstart[dr[i] & 0xFFu] + (dr[i] >> 8)] = (uint32_t)(t0 + i * 64 + lane);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int j = tid + r * SC_THREADS;
        if (j < tile_n && gpos[r] != 0xFFFFFFFFu) vals_out[T.base + gpos[r]] = sv[j];
    }
}

// Reduction of one value per thread over a block of SS_BT.
template <typename V, typename Op>
__device__ __forceinline__ V ss_block_reduce(V v, V *red, Op op) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off >= 1; off >>= 1) v = op(v, (V)__shfl_xor(v, off));
    if (lane == 0) red[wave] = v;
    __syncthreads();
    V r = red[0];
    for (int w = 1; w < SS_BT / 64; ++w) r = op(r, red[w]);
    __syncthreads();
    return r;
}

template <bool VAR>
__global__ void __launch_bounds__(SS_BT)
ss_bucket_sort(const uint64_t *__restrict__ bkeys, const uint32_t *__restrict__ bvals,
               const uint32_t *__restrict__ totals, const uint32_t *__restrict__ bstart,
               const uint64_t *__restrict__ split, SortLayout L, uint64_t *__restrict__ keys_out,
               uint32_t *__restrict__ perm_out, uint32_t *__restrict__ rank_out, double *__restrict__ xs_out,
               int *__restrict__ flag) {
    __shared__ uint64_t sk[SS_CAP];
    __shared__ uint16_t spos[SS_CAP];          // position of the key in the bucket's input
    __shared__ uint16_t sstart[SS_SUB];
    __shared__ uint32_t cursor[SS_SUB / 2];   // two 16-bit counters per word (sub-buckets 2i, 2i+1)
    __shared__ uint64_t red64[SS_BT / 64];
    __shared__ uint32_t red32[SS_BT / 64];
    __shared__ int too_big;
    const int s = blockIdx.y, b = blockIdx.x, tid = threadIdx.x;
    const uint32_t size = totals[(int64_t)s * SS_B + b];
    if (size == 0) return;
    if (size > (uint32_t)SS_CAP) {
        if (tid == 0) *flag = 1;
        return;
    }
    int64_t sbase, sn, tile0;
    int nblk, qrow;
    seg_ref<VAR>(L, s, sbase, sn, tile0, nblk, qrow);
    const uint32_t start = bstart[(int64_t)s * SS_B + b];
    const int64_t base = sbase + start;
    for (int i = tid; i < SS_SUB / 2; i += SS_BT) cursor[i] = 0;
    if (tid == 0) too_big = 0;
    // keys and their particles, both read in order
    uint64_t k[SS_IT];
    uint32_t v[SS_IT];
#pragma unroll
    for (int i = 0; i < SS_IT; ++i) {
        const uint32_t idx = (uint32_t)tid + (uint32_t)i * SS_BT;
        k[i] = idx < size ? bkeys[base + idx] : ~0ull;
        v[i] = idx < size ? bvals[base + idx] : 0u;
    }
    // bounds of the bucket's values: its splitters inside, its extremes at
    // the two ends of the ensemble
    uint64_t kmin, kmax;
    if (b > 0 && b < ss_buckets(sn) - 1) {
        kmin = split[(int64_t)s * SS_B + b];
        kmax = split[(int64_t)s * SS_B + b + 1];
    } else {
        kmin = ~0ull;
        kmax = 0ull;
#pragma unroll
        for (int i = 0; i < SS_IT; ++i)
            if ((uint32_t)tid + (uint32_t)i * SS_BT < size) {
                kmin = k[i] < kmin ? k[i] : kmin;
                kmax = k[i] > kmax ? k[i] : kmax;
            }
        kmin = ss_block_reduce<uint64_t>(kmin, red64, [](uint64_t a, uint64_t c) { return a < c ? a : c; });
        kmax = ss_block_reduce<uint64_t>(kmax, red64, [](uint64_t a, uint64_t c) { return a > c ? a : c; });
    }
    // value sub-buckets: floor((x - lo) SS_SUB / (hi - lo)) is non-decreasing
    // in x (every rounded operation is), so they keep the order; equal values
    // share one.  Bounds that are not finite put every key in one.
    const double lo = value_of(kmin), hi = value_of(kmax);
    const double span = hi - lo;
    const double scale = (span > 0.0 && span <= 1.79e308) ? (double)SS_SUB / span : 0.0;
    __syncthreads();
    uint16_t sub[SS_IT];
#pragma unroll
    for (int i = 0; i < SS_IT; ++i) {
        sub[i] = 0;
        if ((uint32_t)tid + (uint32_t)i * SS_BT < size) {
            const double t = (value_of(k[i]) - lo) * scale;
            sub[i] = (uint16_t)(t >= (double)SS_SUB ? SS_SUB - 1 : (t > 0.0 ? (int)t : 0));
            atomicAdd(&cursor[sub[i] >> 1], 1u << (16 * (sub[i] & 1)));
        }
    }
    __syncthreads();
    // exclusive scan of the sub-bucket counts (two per thread), their maximum
    {
        const uint32_t w0 = cursor[tid];
        const uint32_t c0 = w0 & 0xFFFFu, c1 = w0 >> 16;
        if (c0 > (uint32_t)SS_SUBMAX || c1 > (uint32_t)SS_SUBMAX) too_big = 1;
        const uint32_t c = c0 + c1;
        const int lane = tid & 63, wave = tid >> 6;
        uint32_t inc = c;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t t = __shfl_up(inc, off);
            if (lane >= off) inc += t;
        }
        if (lane == 63) red32[wave] = inc;
        __syncthreads();
        uint32_t pre = 0;
        for (int w = 0; w < wave; ++w) pre += red32[w];
        const uint32_t e0 = pre + inc - c, e1 = e0 + c0;
        sstart[2 * tid] = (uint16_t)e0;
        sstart[2 * tid + 1] = (uint16_t)e1;
        cursor[tid] = e0 | (e1 << 16);
        __syncthreads();
    }
    if (too_big) {
        if (tid == 0) *flag = 1;
        return;
    }
    // every slot first (the atomics of all items in flight together), then
    // the stores
    uint16_t slot[SS_IT];
#pragma unroll
    for (int i = 0; i < SS_IT; ++i) {
        const uint32_t idx = (uint32_t)tid + (uint32_t)i * SS_BT;
        slot[i] = 0xFFFF;
        if (idx < size) {
            const uint32_t sh = 16 * (sub[i] & 1);
            slot[i] = (uint16_t)((atomicAdd(&cursor[sub[i] >> 1], 1u << sh) >> sh) & 0xFFFFu);
        }
    }
#pragma unroll
    for (int i = 0; i < SS_IT; ++i)
        if (slot[i] != 0xFFFF) {
            sk[slot[i]] = k[i];
            spos[slot[i]] = (uint16_t)((uint32_t)tid + (uint32_t)i * SS_BT);
        }
    __syncthreads();
    // place: the keys of the sub-bucket before this one by (key, particle)
    uint16_t fin[SS_IT];
#pragma unroll
    for (int i = 0; i < SS_IT; ++i) {
        const uint32_t idx = (uint32_t)tid + (uint32_t)i * SS_BT;
        fin[i] = 0xFFFF;
        if (idx < size) {
            const uint32_t a = sstart[sub[i]], e = (cursor[sub[i] >> 1] >> (16 * (sub[i] & 1))) & 0xFFFFu;
            const uint32_t me = slot[i];
            // four entries per step, their LDS loads in flight together; the
            // steps past the end read the key's own slot, which never counts.
            // Positions are read only for equal keys in other slots.
            uint32_t r = a;
            for (uint32_t j = a; j < e; j += 4) {
                uint64_t kj[4];
                uint32_t jj[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    jj[u] = j + u < e ? j + u : me;
                    kj[u] = sk[jj[u]];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (kj[u] < k[i]) ++r;
                    else if (kj[u] == k[i] && jj[u] != me && bvals[base + spos[jj[u]]] < v[i]) ++r;
                }
            }
            fin[i] = (uint16_t)r;
        }
    }
    // the keys, then their particles, pass through LDS to their final
    // slots and leave in order (the particles in the keys' own array)
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SS_IT; ++i)
        if (fin[i] != 0xFFFF) sk[fin[i]] = k[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SS_IT; ++i) {
        const uint32_t idx = (uint32_t)tid + (uint32_t)i * SS_BT;
        if (idx < size) {
            const uint64_t ok = sk[idx];
            keys_out[base + idx] = ok;
            if (xs_out) xs_out[base + idx] = value_of(ok);
        }
    }
    if (!perm_out && !rank_out) return;
    __syncthreads();
    uint32_t *sv = reinterpret_cast<uint32_t *>(sk);
#pragma unroll
    for (int i = 0; i < SS_IT; ++i)
        if (fin[i] != 0xFFFF) sv[fin[i]] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SS_IT; ++i) {
        const uint32_t idx = (uint32_t)tid + (uint32_t)i * SS_BT;
        if (idx < size) {
            const uint32_t op = sv[idx];
            if (perm_out) perm_out[base + idx] = op;
            if (rank_out) rank_out[sbase + op] = start + idx;
        }
    }
}

// ---------------------------------------------------------------------------
// Fix-up after the passes over the high 32 bits of 64-bit keys.  The keys
// are then ordered by their high halves, and among equal high halves by
// particle (the passes are stable), so a run of equal high halves needs
// only its own order by the full key, ties by position.  Every key finds the
// run around it in the tile's keys (staged in LDS with FIX_MAX + 1 keys on
// either side), counts the keys of the run that precede it in that order,
// and goes to its final place with the rank, perm and sorted-value outputs
// of the last pass.  A run longer than FIX_MAX sets *flag: the complete sort
// then runs (guarded by the flag) and redoes every output.
// ---------------------------------------------------------------------------
constexpr int FIX_MAX = 64;
constexpr int FIX_HALO = FIX_MAX + 1;

template <bool VAR, bool PAYLOAD>
__global__ void __launch_bounds__(RS_THREADS)
rs_fixup(const uint64_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in, uint64_t *__restrict__ keys_out,
         SortLayout L, uint32_t *__restrict__ rank_out, uint32_t *__restrict__ perm_out, double *__restrict__ xs_out,
         int *__restrict__ flag) {
    constexpr int TILE = RS_THREADS * RS_ITEMS;
    __shared__ uint64_t sk[TILE + 2 * FIX_HALO];
    if (L.guard && *L.guard == 0) return;
    const TileRef T = tile_ref<VAR>(L, xcd_tile(blockIdx.x, gridDim.x));
    const uint64_t *k = keys_in + T.base;
    const int64_t n = T.n, t0 = (int64_t)T.blk * TILE;
    // sk[j] = k[t0 - FIX_HALO + j] where that position exists; all loads
    // first, so that they are in flight together
    constexpr int SK = TILE + 2 * FIX_HALO, SK_PER = (SK + RS_THREADS - 1) / RS_THREADS;
    uint64_t ld[SK_PER];
#pragma unroll
    for (int r = 0; r < SK_PER; ++r) {
        const int j = (int)threadIdx.x + r * RS_THREADS;
        const int64_t q = t0 - FIX_HALO + j;
        ld[r] = (j < SK && q >= 0 && q < n) ? k[q] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < SK_PER; ++r) {
        const int j = (int)threadIdx.x + r * RS_THREADS;
        if (j < SK) sk[j] = ld[r];
    }
    __syncthreads();
    bool too_long = false;
    // final places first, then all stores of the tile's keys at once
    int64_t pos[RS_ITEMS];
    uint64_t key[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t p = t0 + (int64_t)i * RS_THREADS + threadIdx.x;
        pos[i] = -1;
        key[i] = 0;
        if (p < n) {
            const int j = (int)(p - t0) + FIX_HALO;  // p in sk
            const uint64_t kp = sk[j];
            const uint32_t hp = (uint32_t)(kp >> 32);
            // the run [p - back, p + fwd] of equal high halves, at most FIX_MAX long
            int back = 0, fwd = 0;
            while (back < FIX_MAX && p - back > 0 && (uint32_t)(sk[j - back - 1] >> 32) == hp) ++back;
            while (fwd < FIX_MAX && p + fwd + 1 < n && (uint32_t)(sk[j + fwd + 1] >> 32) == hp) ++fwd;
            key[i] = kp;
            if (back + fwd + 1 > FIX_MAX) {
                too_long = true;
            } else if (back + fwd == 0) {
                pos[i] = p;
            } else {
                int r = 0;
                for (int b = -back; b <= fwd; ++b) {
                    const uint64_t kb = sk[j + b];
                    r += (kb < kp || (kb == kp && b < 0)) ? 1 : 0;
                }
                pos[i] = p - back + r;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        if (pos[i] >= 0) {
            keys_out[T.base + pos[i]] = key[i];
            if (xs_out) xs_out[T.base + pos[i]] = value_of(key[i]);
        }
    }
    if constexpr (PAYLOAD) {
        uint32_t val[RS_ITEMS];
#pragma unroll
        for (int i = 0; i < RS_ITEMS; ++i)
            val[i] = pos[i] >= 0 ? vals_in[T.base + t0 + (int64_t)i * RS_THREADS + threadIdx.x] : 0u;
#pragma unroll
        for (int i = 0; i < RS_ITEMS; ++i) {
            if (pos[i] >= 0) {
                if (rank_out && (int64_t)val[i] < n) rank_out[T.base + val[i]] = (uint32_t)pos[i];
                if (perm_out) perm_out[T.base + pos[i]] = val[i];
            }
        }
    }
    if (too_long) *flag = 1;
}

// ---------------------------------------------------------------------------
// Ranks from the permutation (sorted position -> particle) without stores to
// random addresses: a 4-byte store at a random index leaves its cache line
// partly written, and the line then costs a whole memory sector.  Instead
//   rs_rank_bucket  every tile of the permutation groups its (position,
//                   particle) pairs by the block of TILE particles the
//                   particle belongs to and appends each group, as one
//                   contiguous run, to that block's region of a staging
//                   buffer (the region has one slot per particle of the
//                   block; a cursor per block hands out the slots),
//   rs_rank_place   every block of TILE particles takes its region, places
//                   the ranks in LDS and writes them out in particle order.
// A pair packs the position (below 2^20) and the particle's offset in its
// block (below 2^12) into 32 bits, so segments of up to 2^20 keys take this
// path.  Both kernels return at once where the fix-up raised its flag (the
// complete sort then writes the ranks).
// ---------------------------------------------------------------------------
constexpr int RK_SHIFT = 12;
constexpr int64_t RK_MAX_N = (int64_t)1 << 20;
static_assert((1 << RK_SHIFT) == RS_THREADS * RS_ITEMS, "a block of particles is one tile");
static_assert(RS_THREADS == RS_RADIX, "one thread per particle block of a segment");

template <bool VAR>
__global__ void __launch_bounds__(RS_THREADS)
rs_rank_bucket(const uint32_t *__restrict__ perm, SortLayout L, uint32_t *__restrict__ cursor,
               uint32_t *__restrict__ staged, const int *__restrict__ flag) {
    constexpr int TILE = RS_THREADS * RS_ITEMS;
    __shared__ uint32_t cnt[RS_RADIX], lofs[RS_RADIX], gofs[RS_RADIX], wtot[RS_WAVES];
    __shared__ uint32_t stage[TILE];
    __shared__ uint8_t sblk[TILE];
    if ((L.guard && *L.guard == 0) || *flag != 0) return;
    const TileRef T = tile_ref<VAR>(L, xcd_tile(blockIdx.x, gridDim.x));
    const int tid = threadIdx.x;
    cnt[tid] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)T.blk * TILE;
    uint32_t p[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t pos = t0 + (int64_t)i * RS_THREADS + tid;
        p[i] = pos < T.n ? perm[T.base + pos] : 0xFFFFFFFFu;
    }
    uint32_t slot[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i)
        if ((int64_t)p[i] < T.n) slot[i] = atomicAdd(&cnt[p[i] >> RK_SHIFT], 1u);
    __syncthreads();
    const uint32_t c = cnt[tid];
    lofs[tid] = block_exclusive_256(c, wtot);
    if (c != 0) gofs[tid] = atomicAdd(&cursor[T.tile0 + tid], c);  // c != 0 only for blocks of this segment
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        if ((int64_t)p[i] < T.n) {
            const uint32_t b = p[i] >> RK_SHIFT, j = lofs[b] + slot[i];
            const uint32_t pos = (uint32_t)(t0 + i * RS_THREADS + tid);
            stage[j] = (pos << RK_SHIFT) | (p[i] & (TILE - 1));
            sblk[j] = (uint8_t)b;
        }
    }
    __syncthreads();
    const uint32_t total = lofs[RS_RADIX - 1] + cnt[RS_RADIX - 1];
    for (uint32_t j = tid; j < total; j += RS_THREADS) {
        const uint32_t b = sblk[j];
        const int64_t b0 = (int64_t)b << RK_SHIFT;
        const int64_t bn = T.n - b0 < TILE ? T.n - b0 : TILE;
        const uint32_t s = gofs[b] + (j - lofs[b]);
        if ((int64_t)s < bn) staged[T.base + b0 + s] = stage[j];
    }
}

template <bool VAR>
__global__ void __launch_bounds__(RS_THREADS)
rs_rank_place(const uint32_t *__restrict__ staged, SortLayout L, uint32_t *__restrict__ rank_out,
              const int *__restrict__ flag) {
    constexpr int TILE = RS_THREADS * RS_ITEMS;
    __shared__ uint32_t r[TILE];
    if ((L.guard && *L.guard == 0) || *flag != 0) return;
    const TileRef T = tile_ref<VAR>(L, xcd_tile(blockIdx.x, gridDim.x));
    const int64_t b0 = (int64_t)T.blk * TILE;
    const int bn = (int)(T.n - b0 < TILE ? T.n - b0 : TILE);
    uint32_t e[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int j = i * RS_THREADS + threadIdx.x;
        e[i] = j < bn ? staged[T.base + b0 + j] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i)
        if (i * RS_THREADS + (int)threadIdx.x < bn && (int)(e[i] & (TILE - 1)) < bn) r[e[i] & (TILE - 1)] = e[i] >> RK_SHIFT;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int j = i * RS_THREADS + threadIdx.x;
        if (j < bn) rank_out[T.base + b0 + j] = r[j];
    }
}

// ---------------------------------------------------------------------------
// Knots (midpoint convention) from the sorted keys; moment totals.
// ---------------------------------------------------------------------------
template <typename K, bool VAR>
__global__ void rs_knots(const K *__restrict__ sorted, SortLayout L, int nq, double *__restrict__ q) {
#pragma clang fp contract(off)
    if (L.guard && *L.guard == 0) return;
    int64_t base, n, tile0;
    int nblk, qrow;
    seg_ref<VAR>(L, blockIdx.x, base, n, tile0, nblk, qrow);
    const K *s = sorted + base;
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
        q[(int64_t)qrow * (nq + 1) + j] = v;
    }
}

template <bool VAR>
__global__ void rs_moments(const double *__restrict__ part, SortLayout L, double *__restrict__ mom) {
    if (L.guard && *L.guard == 0) return;
    int64_t base, n, tile0;
    int nblk, qrow;
    seg_ref<VAR>(L, blockIdx.x, base, n, tile0, nblk, qrow);
    const int lane = threadIdx.x;  // one wave
    for (int m = 0; m < 4; ++m) {
        double s = 0;
        for (int b = lane; b < nblk; b += 64) s += part[(tile0 + b) * 4 + m];
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) mom[(int64_t)qrow * 4 + m] = s / (double)n;
    }
}

__global__ void zero_u32(uint32_t *p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---------------------------------------------------------------------------
// Knots of matched ensembles from the sort of their priors.
//
// Matching moves every prior value by a smooth function of its rank, so the
// matched values taken in the prior's rank order, z_r = M(xs_r) (xs the
// sorted prior), are nearly sorted.  A position c is a cut where every z
// before it is below every z from it on, in key order (c = 0 and c = n are
// cuts); between neighbouring cuts a <= r < b the order statistics of ranks
// a..b-1 are z_a..z_{b-1} sorted.  The order statistic of rank r is thus the
// key of rank r - a among the few values between the cuts around r.  The
// maxima before and minima after every chunk of 64 ranks come from one
// streaming pass and a scan; inside a chunk, from wave scans.
// ---------------------------------------------------------------------------
constexpr int MK_REACH = 8;  // chunks searched on either side of a rank for a cut

template <typename K>
__device__ __forceinline__ K shfl_key(K v, int src) {
    return (K)__shfl((unsigned long long)v, src);
}

// Key of the matched value of the prior with key kp at rank r.
template <typename K>
__device__ __forceinline__ K matched_key(K kp, int64_t r, const double *dk, double nd, double Q) {
    using V = typename KeyTraits<K>::V;
    return key_of(matched_value<V>((V)value_of(kp), (uint64_t)r, dk, nd, Q));
}

// Arguments of the matched-knot kernels.  Equal lengths (segs == NULL):
// ensemble s holds keys [s n, s n + n) and knot rows s of qt, qp (strides
// qts, qps) and q.  Unequal lengths: the segment table.
struct MkArgs {
    const void *sorted;  // the sorted keys
    int64_t n, nch, ngr;  // equal lengths: ranks, chunks, groups per ensemble
    const double *qt, *qp;
    int64_t qts, qps;
    double *q;
    const MkSeg *segs;
    const int *group_seg;
    void *pre, *suf, *gx, *gn;  // extremes: [chunks], [chunks], [groups], [groups]
    int nq;
    int *flag;     // raised where some ensemble's knots need the sort
    int *segflag;  // unequal lengths: one flag per ensemble, or NULL
};

// One ensemble as the kernels see it.
struct MkRef {
    int64_t base, n, nch, ngr, ch0, gr0;
    const double *qt, *qp;
    double *q;
};

template <bool VAR>
__device__ __forceinline__ MkRef mk_ref(const MkArgs &A, int s) {
    MkRef R;
    if constexpr (VAR) {
        const MkSeg g = A.segs[s];
        R.base = g.base;
        R.n = g.n;
        R.nch = (g.n + 63) / 64;
        R.ngr = (R.nch + 63) / 64;
        R.ch0 = g.ch0;
        R.gr0 = g.gr0;
        R.qt = A.qt + (int64_t)g.qt_row * (A.nq + 1);
        R.qp = A.qp + (int64_t)g.qp_row * (A.nq + 1);
        R.q = A.q + (int64_t)g.q_row * (A.nq + 1);
    } else {
        R.base = s * A.n;
        R.n = A.n;
        R.nch = A.nch;
        R.ngr = A.ngr;
        R.ch0 = s * A.nch;
        R.gr0 = s * A.ngr;
        R.qt = A.qt + s * A.qts;
        R.qp = A.qp + s * A.qps;
        R.q = A.q + (int64_t)s * (A.nq + 1);
    }
    return R;
}

__device__ __forceinline__ void load_dk(double *dk, const MkRef &R, int nq) {
    for (int j = threadIdx.x; j <= nq; j += blockDim.x) dk[j] = R.qt[j] - R.qp[j];
    __syncthreads();
}

// Chunk and group extremes.  A group is 64 chunks (4096 ranks, one block of
// 256 threads, 4 consecutive ranks per thread and pass).  For every chunk c
// of group g: pre[c] = largest key of the chunks of g before c, suf[c] =
// smallest key of the chunks of g from c on; gx[g], gn[g] = largest and
// smallest key of g (turned into the values over the groups before g and
// from g on by mk_scan).
constexpr int MK_GROUP = 64;

template <typename K, bool VAR>
__global__ void __launch_bounds__(256) mk_extremes(MkArgs A) {
    extern __shared__ double dk[];
    __shared__ K cx[MK_GROUP], cn[MK_GROUP];
    int seg;
    int64_t g;
    if constexpr (VAR) {
        seg = A.group_seg[blockIdx.x];
        g = (int64_t)blockIdx.x - A.segs[seg].gr0;
    } else {
        seg = blockIdx.y;
        g = blockIdx.x;
    }
    const MkRef R = mk_ref<VAR>(A, seg);
    load_dk(dk, R, A.nq);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const K *sorted = (const K *)A.sorted + R.base;
    const int64_t n = R.n;
    const double nd = (double)n, Q = (double)A.nq;
    // all sixteen loads of a thread first, so that they are in flight together
    K v[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t e0 = g * (MK_GROUP * 64) + w * 1024 + i * 256 + 4 * lane;
#pragma unroll
        for (int t = 0; t < 4; ++t) v[i][t] = e0 + t < n ? sorted[e0 + t] : (K)0;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        // ranks e0..e0+3 of chunk 16 w + 4 i + lane / 16 of the group
        const int64_t e0 = g * (MK_GROUP * 64) + w * 1024 + i * 256 + 4 * lane;
        K kx = 0, kn = ~(K)0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (e0 + t < n) {
                const K z = matched_key<K>(v[i][t], e0 + t, dk, nd, Q);
                kx = z > kx ? z : kx;
                kn = z < kn ? z : kn;
            }
        }
        for (int off = 1; off < 16; off <<= 1) {  // over the 16 lanes of the chunk
            const K ox = (K)__shfl_xor((unsigned long long)kx, off), on = (K)__shfl_xor((unsigned long long)kn, off);
            kx = ox > kx ? ox : kx;
            kn = on < kn ? on : kn;
        }
        if ((lane & 15) == 0) {
            cx[w * 16 + i * 4 + (lane >> 4)] = kx;
            cn[w * 16 + i * 4 + (lane >> 4)] = kn;
        }
    }
    __syncthreads();
    if (w == 0) {
        // lane = chunk of the group: exclusive prefix max, inclusive suffix min
        const K x = cx[lane], m = cn[lane];
        K px = x, sn = m;
        for (int off = 1; off < 64; off <<= 1) {
            const K u = shfl_key(px, lane >= off ? lane - off : lane);
            const K d = shfl_key(sn, lane + off < 64 ? lane + off : lane);
            px = u > px ? u : px;
            sn = d < sn ? d : sn;
        }
        K ex = shfl_key(px, lane > 0 ? lane - 1 : 0);
        if (lane == 0) ex = 0;
        const int64_t c = g * MK_GROUP + lane;
        if (c < R.nch) {
            ((K *)A.pre)[R.ch0 + c] = ex;
            ((K *)A.suf)[R.ch0 + c] = sn;
        }
        if (lane == 63) ((K *)A.gx)[R.gr0 + g] = px;
        if (lane == 0) ((K *)A.gn)[R.gr0 + g] = sn;
    }
}

// Per ensemble (one block of 256): gx[g] <- largest key of the groups before
// g, gn[g] <- smallest key of the groups from g on.
template <typename K, bool VAR>
__global__ void __launch_bounds__(256) mk_scan(MkArgs A) {
    __shared__ K wmx[4], wmn[4];
    const MkRef R = mk_ref<VAR>(A, blockIdx.x);
    const int64_t ngr = R.ngr;
    K *gx = (K *)A.gx + R.gr0, *gn = (K *)A.gn + R.gr0;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t per = (ngr + 255) / 256;
    const int64_t g0 = tid * per < ngr ? tid * per : ngr, g1 = g0 + per < ngr ? g0 + per : ngr;
    K lx = 0, ln = ~(K)0;
    for (int64_t g = g0; g < g1; ++g) {
        lx = gx[g] > lx ? gx[g] : lx;
        ln = gn[g] < ln ? gn[g] : ln;
    }
    K px = lx, sn = ln;
    for (int off = 1; off < 64; off <<= 1) {
        const K u = shfl_key(px, lane >= off ? lane - off : lane);
        const K d = shfl_key(sn, lane + off < 64 ? lane + off : lane);
        px = u > px ? u : px;
        sn = d < sn ? d : sn;
    }
    if (lane == 63) wmx[w] = px;
    if (lane == 0) wmn[w] = sn;
    __syncthreads();
    K ex = shfl_key(px, lane > 0 ? lane - 1 : 0);
    if (lane == 0) ex = 0;
    K es = shfl_key(sn, lane < 63 ? lane + 1 : 63);
    if (lane == 63) es = ~(K)0;
    for (int k = 0; k < 4; ++k) {
        if (k < w) ex = wmx[k] > ex ? wmx[k] : ex;
        if (k > w) es = wmn[k] < es ? wmn[k] : es;
    }
    for (int64_t g = g0; g < g1; ++g) {
        const K v = gx[g];
        gx[g] = ex;
        ex = v > ex ? v : ex;
    }
    for (int64_t g = g1 - 1; g >= g0; --g) {
        es = gn[g] < es ? gn[g] : es;
        gn[g] = es;
    }
}

// The extremes one ensemble's cut tests read.
template <typename K>
struct MkExt {
    const K *pre, *suf, *gx, *gn;
    int64_t nch, ngr;
    // largest key of the chunks before c
    __device__ K before(int64_t c) const {
        const K a = pre[c], b = gx[c / MK_GROUP];
        return a > b ? a : b;
    }
    // smallest key of the chunks from c on (c <= nch)
    __device__ K from(int64_t c) const {
        if (c >= nch) return ~(K)0;
        const int64_t g = c / MK_GROUP;
        const K a = suf[c], b = g + 1 < ngr ? gn[g + 1] : ~(K)0;
        return a < b ? a : b;
    }
};

// Cut flags of the positions 64c + lane of chunk c (the wave).
template <typename K>
__device__ __forceinline__ uint64_t chunk_cuts(const K *sorted, int64_t n, const MkExt<K> &E, int64_t c,
                                               const double *dk, double nd, double Q, int lane) {
    const int64_t p = c * 64 + lane;
    K kx = 0, kn = ~(K)0;
    if (p < n) {
        kx = matched_key<K>(sorted[p], p, dk, nd, Q);
        kn = kx;
    }
    K px = kx, sn = kn;  // inclusive prefix max, inclusive suffix min inside the chunk
    for (int off = 1; off < 64; off <<= 1) {
        const K u = shfl_key(px, lane >= off ? lane - off : lane);
        const K d = shfl_key(sn, lane + off < 64 ? lane + off : lane);
        px = u > px ? u : px;
        sn = d < sn ? d : sn;
    }
    K before = shfl_key(px, lane > 0 ? lane - 1 : 0);
    if (lane == 0) before = 0;
    const K b0 = E.before(c);
    before = b0 > before ? b0 : before;
    const K a0 = E.from(c + 1);
    const K from = a0 < sn ? a0 : sn;
    const bool cut = p == 0 || p == n || (p < n && before <= from);
    return __ballot(cut);
}

// Key of the order statistic of rank r (the wave); sets *flag (and the
// ensemble's flag when there is one) where the cuts around r are not found
// within MK_REACH chunks or lie more than 64 ranks apart.
template <typename K>
__device__ K order_stat(const K *sorted, int64_t n, const MkExt<K> &E, int64_t r, const double *dk, double nd,
                        double Q, int lane, int *flag, int *segflag) {
    const int64_t nch = E.nch;
    const int64_t c = r / 64;
    const int off = (int)(r - c * 64);
    const uint64_t mc = chunk_cuts<K>(sorted, n, E, c, dk, nd, Q, lane);
    int64_t a = -1, b = -1;
    uint64_t m = mc & (off == 63 ? ~0ull : ((2ull << off) - 1));  // positions <= r
    if (m) a = c * 64 + 63 - __builtin_clzll(m);
    for (int64_t cc = c - 1; a < 0 && cc >= 0 && cc >= c - MK_REACH; --cc) {
        m = chunk_cuts<K>(sorted, n, E, cc, dk, nd, Q, lane);
        if (m) a = cc * 64 + 63 - __builtin_clzll(m);
    }
    m = off == 63 ? 0ull : mc & ~((2ull << off) - 1);  // positions > r
    if (m) b = c * 64 + __builtin_ctzll(m);
    for (int64_t cc = c + 1; b < 0 && cc <= c + MK_REACH; ++cc) {
        if (cc >= nch) {
            b = n;
            break;
        }
        m = chunk_cuts<K>(sorted, n, E, cc, dk, nd, Q, lane);
        if (m) b = cc * 64 + __builtin_ctzll(m);
    }
    if (a < 0 || b < 0 || b - a > 64) {
        if (lane == 0) {
            *flag = 1;
            if (segflag) *segflag = 1;
        }
        return 0;
    }
    // rank r - a among z_a..z_{b-1}: count the smaller keys (ties by position)
    const int ms = (int)(b - a);
    const K w = lane < ms ? matched_key<K>(sorted[a + lane], a + lane, dk, nd, Q) : ~(K)0;
    int below = 0;
    for (int l = 0; l < ms; ++l) {
        const K o = shfl_key(w, l);
        below += (o < w || (o == w && l < lane)) ? 1 : 0;
    }
    const uint64_t sel = __ballot(lane < ms && below == (int)(r - a));
    return shfl_key(w, __builtin_ctzll(sel));
}

// Midpoint (Hazen) knots of every matched ensemble, the arithmetic of
// rs_knots on the order statistics: one wave per knot.
template <typename K, bool VAR>
__global__ void __launch_bounds__(256) mk_knots(MkArgs A) {
#pragma clang fp contract(off)
    extern __shared__ double dk[];
    const MkRef R = mk_ref<VAR>(A, blockIdx.y);
    load_dk(dk, R, A.nq);
    const int nq = A.nq;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j > nq) return;
    const int lane = threadIdx.x & 63;
    const int64_t n = R.n;
    const K *sorted = (const K *)A.sorted + R.base;
    const MkExt<K> E{(const K *)A.pre + R.ch0, (const K *)A.suf + R.ch0, (const K *)A.gx + R.gr0,
                     (const K *)A.gn + R.gr0, R.nch, R.ngr};
    int *flag = A.flag;
    int *segflag = (VAR && A.segflag) ? A.segflag + blockIdx.y : nullptr;
    const double nd = (double)n, Q = (double)nq;
    const double t = (double)((int64_t)j * n) / (double)nq - 0.5;
    double v;
    if (t <= 0.0) {
        v = value_of(order_stat<K>(sorted, n, E, 0, dk, nd, Q, lane, flag, segflag));
    } else if (t >= (double)(n - 1)) {
        v = value_of(order_stat<K>(sorted, n, E, n - 1, dk, nd, Q, lane, flag, segflag));
    } else {
        const int64_t r = (int64_t)floor(t);
        const double f = t - (double)r;
        const double a = value_of(order_stat<K>(sorted, n, E, r, dk, nd, Q, lane, flag, segflag));
        const double b = value_of(order_stat<K>(sorted, n, E, r + 1, dk, nd, Q, lane, flag, segflag));
        v = a + f * (b - a);
        v = v < b ? v : b;
    }
    if (lane == 0) R.q[j] = v;
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int64_t sort_tiles(int64_t n) {
    const int64_t tile = (int64_t)RS_THREADS * RS_ITEMS;
    return (n + tile - 1) / tile;
}

size_t sort_ws_bytes(int64_t total_keys, int64_t total_tiles, int nseg, int precision, bool payload) {
    const size_t ks = precision == PR_F32 ? 4 : 8;
    size_t b = align256(total_keys * ks) * 2 + align256((size_t)total_tiles * RS_RADIX * 4) +
               align256((size_t)nseg * RS_RADIX * 4) + align256((size_t)total_tiles * 4 * 8) + 256 + 256 +
               align256((size_t)nseg * SS_B * (8 + 4 + 8 * SS_RUNS));
    if (payload) b += align256(total_keys * 4) * 2;
    return b;
}

bool splitter_sorts(int64_t n) { return n >= SS_MIN_N && n <= SS_MAX_N; }

size_t restrict_ws(int64_t n, int k, int precision) {
    return sort_ws_bytes((int64_t)n * k, sort_tiles(n) * k, k, precision, true);
}

template <typename K, bool VAR>
static int sort_impl(const void *x, const SortLayout &L, int64_t total_keys, int64_t total_tiles, int nq,
                     const pr_grid *hg, double *q, uint32_t *rank, uint32_t *perm, double *xs, double *mom,
                     uint32_t *hist, void *ws, hipStream_t st) {
    constexpr int ITEMS = RS_ITEMS;
    const bool payload = rank || perm;
    char *p = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    K *keys[2];
    uint32_t *vals[2] = {nullptr, nullptr};
    keys[0] = (K *)p; p += align256(total_keys * sizeof(K));
    keys[1] = (K *)p; p += align256(total_keys * sizeof(K));
    uint32_t *counts = (uint32_t *)p; p += align256((size_t)total_tiles * RS_RADIX * 4);
    uint32_t *totals = (uint32_t *)p; p += align256((size_t)L.nseg * RS_RADIX * 4);
    double *mom_part = (double *)p; p += align256((size_t)total_tiles * 4 * 8);
    if (payload) {
        vals[0] = (uint32_t *)p; p += align256(total_keys * 4);
        vals[1] = (uint32_t *)p;
    }
    HistArgs ha{hist, 0, 0.0, 0.0};
    size_t cell_lds = 0;
    if (hist) {
        ha.cells = hg->n_cells;
        ha.lo = hg->x_lo;
        ha.inv_h = (double)hg->n_cells / (hg->x_hi - hg->x_lo);
        cell_lds = (size_t)hg->n_cells * 4;
        const int64_t cnt = (int64_t)L.nseg * hg->n_cells;
        const int64_t blocks = (cnt + 255) / 256 < 1024 ? (cnt + 255) / 256 : 1024;
        hipLaunchKernelGGL(zero_u32, dim3((unsigned)blocks), dim3(256), 0, st, hist, cnt);
        PR_LAUNCHED();
    }
    int *flag = (int *)p;  // 256 bytes after the payload (or the moment) buffers
    if (payload) flag = (int *)((char *)vals[1] + align256(total_keys * 4));
    uint64_t *split = (uint64_t *)((char *)flag + 256);  // splitters, [nseg][SS_B]
    uint32_t *bstart = (uint32_t *)(split + (size_t)L.nseg * SS_B);  // bucket starts, [nseg][SS_B]
    uint64_t *runq = (uint64_t *)(bstart + (size_t)L.nseg * SS_B);  // run quantiles, [nseg][SS_RUNS][SS_B]
    const dim3 grid((unsigned)total_tiles);
    const dim3 rows((unsigned)(((int64_t)L.nseg * RS_RADIX + 3) / 4));
    // outputs of the last pass (the ranks move to the staging kernels below
    // where they take over)
    uint32_t *rank_last = rank, *perm_last = perm;
    const int64_t max_n = VAR ? L.max_n : L.n;
    const bool staged_ranks = rank != nullptr && max_n > 0 && max_n <= RK_MAX_N;
    // ranks from the permutation in order, through the staging buffer
    auto stage_ranks = [&](const uint32_t *perm_in, uint32_t *staging) -> int {
        const int64_t zb = (total_tiles + 255) / 256 < 1024 ? (total_tiles + 255) / 256 : 1024;
        hipLaunchKernelGGL(zero_u32, dim3((unsigned)zb), dim3(256), 0, st, counts, total_tiles);
        PR_LAUNCHED();
        hipLaunchKernelGGL((rs_rank_bucket<VAR>), grid, dim3(RS_THREADS), 0, st, perm_in, L, counts, staging,
                           (const int *)flag);
        PR_LAUNCHED();
        hipLaunchKernelGGL((rs_rank_place<VAR>), grid, dim3(RS_THREADS), 0, st, (const uint32_t *)staging, L, rank,
                           (const int *)flag);
        PR_LAUNCHED();
        return PR_OK;
    };
    // One LSD pass over the byte at shift: keys[in] -> keys[out] (pass 0
    // reads the values), with the statistics on the first read and the rank,
    // perm and sorted-value outputs on the last pass.
    auto pass = [&](const SortLayout &LL, int shift, bool first, bool last, int in, int out, bool stats) -> int {
        if (first)
            hipLaunchKernelGGL((rs_count<K, ITEMS, true, VAR>), grid, dim3(RS_THREADS), stats ? cell_lds : 0, st, x,
                               shift, LL, counts, (stats && mom) ? mom_part : nullptr,
                               stats ? ha : HistArgs{nullptr, 0, 0.0, 0.0});
        else
            hipLaunchKernelGGL((rs_count<K, ITEMS, false, VAR>), grid, dim3(RS_THREADS), 0, st,
                               (const void *)keys[in], shift, LL, counts, nullptr, HistArgs{nullptr, 0, 0.0, 0.0});
        PR_LAUNCHED();
        if constexpr (VAR)
            hipLaunchKernelGGL((rs_rowscan_seg<VAR>), dim3((unsigned)LL.nseg), dim3(RS_RADIX), 0, st, counts, totals,
                               LL);
        else
            hipLaunchKernelGGL((rs_rowscan<VAR>), rows, dim3(256), 0, st, counts, totals, LL);
        PR_LAUNCHED();
#define PR_SCATTER(FIRST, LAST, PAY, SRC, VIN, VOUT)                                                            \
    hipLaunchKernelGGL((rs_scatter<K, ITEMS, FIRST, LAST, PAY, VAR>), grid, dim3(RS_THREADS), 0, st, SRC, VIN,     \
                       keys[out], VOUT, (const uint32_t *)counts, (const uint32_t *)totals, shift, LL,         \
                       LAST ? rank_last : nullptr, LAST ? perm_last : nullptr, LAST ? xs : nullptr)
        if (payload) {
            if (first) PR_SCATTER(true, false, true, x, nullptr, vals[out]);
            else if (!last) PR_SCATTER(false, false, true, (const void *)keys[in], vals[in], vals[out]);
            else PR_SCATTER(false, true, true, (const void *)keys[in], vals[in], nullptr);
        } else {
            if (first) PR_SCATTER(true, false, false, x, nullptr, nullptr);
            else if (!last) PR_SCATTER(false, false, false, (const void *)keys[in], nullptr, nullptr);
            else PR_SCATTER(false, true, false, (const void *)keys[in], nullptr, nullptr);
        }
#undef PR_SCATTER
        PR_LAUNCHED();
        return PR_OK;
    };
    constexpr int P = KeyTraits<K>::passes;
    // The splitter sort takes FP64 ensembles of SS_MIN_N..SS_MAX_N keys (a
    // segment table says its shortest and longest).
    bool splitter = false;
    if constexpr (std::is_same<K, uint64_t>::value)
        splitter = payload && L.guard == nullptr &&
                   (VAR ? (L.min_n >= SS_MIN_N && L.max_n <= SS_MAX_N) : (L.n >= SS_MIN_N && L.n <= SS_MAX_N));
    if (splitter) {
        if constexpr (std::is_same<K, uint64_t>::value) {
            // the splitter sort, then the complete radix sort guarded by its flag
            hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, st, (uint32_t *)flag, (int64_t)1);
            PR_LAUNCHED();
            hipLaunchKernelGGL((ss_sample_runs<VAR>), dim3(SS_RUNS, (unsigned)L.nseg), dim3(SS_RUN / 2), 0, st,
                               (const double *)x, L, runq);
            PR_LAUNCHED();
            hipLaunchKernelGGL((ss_splitters<VAR>), dim3((unsigned)L.nseg), dim3(SS_B), 0, st,
                               (const uint64_t *)runq, L, split);
            PR_LAUNCHED();
            // the bucket of every key, one byte each, in the first payload
            // buffer (free until the bucket sort writes the permutation)
            uint8_t *bucket = (uint8_t *)vals[0];
            hipLaunchKernelGGL((ss_count<VAR>), grid, dim3(SC_THREADS), cell_lds, st, (const double *)x,
                               (const uint64_t *)split, L, counts, mom ? mom_part : nullptr, ha, bucket);
            PR_LAUNCHED();
            if constexpr (VAR)
                hipLaunchKernelGGL((rs_rowscan_seg<true>), dim3((unsigned)L.nseg), dim3(RS_RADIX), 0, st, counts,
                                   totals, L);
            else
                hipLaunchKernelGGL((rs_rowscan<false>), rows, dim3(256), 0, st, counts, totals, L);
            PR_LAUNCHED();
            hipLaunchKernelGGL((ss_scatter<VAR>), grid, dim3(SC_THREADS), 0, st, (const double *)x,
                               (const uint8_t *)bucket, (uint64_t *)keys[1], vals[1], (const uint32_t *)counts,
                               (const uint32_t *)totals, L, bstart);
            PR_LAUNCHED();
            uint32_t *perm_fix = perm ? perm : (staged_ranks ? vals[0] : nullptr);
            // one block per bucket of the ensemble with the most (the blocks
            // of the others' empty buckets return at once)
            const int nb = ss_buckets(VAR ? L.max_n : L.n);
            hipLaunchKernelGGL((ss_bucket_sort<VAR>), dim3((unsigned)nb, (unsigned)L.nseg), dim3(SS_BT), 0, st,
                               (const uint64_t *)keys[1], (const uint32_t *)vals[1], (const uint32_t *)totals,
                               (const uint32_t *)bstart, (const uint64_t *)split, L, (uint64_t *)keys[0], perm_fix,
                               staged_ranks ? nullptr : rank, xs, flag);
            PR_LAUNCHED();
            if (staged_ranks) PR_CHECK(stage_ranks(perm_fix, vals[1]));
            SortLayout LG = L;
            LG.guard = flag;
            for (int j = 0; j < P; ++j) PR_CHECK(pass(LG, 8 * j, j == 0, j == P - 1, j & 1, (j + 1) & 1, false));
        }
    } else if constexpr (std::is_same<K, uint64_t>::value) {
        // the high 32 bits (passes 4..7, ending in buffer 1), the fix-up of
        // runs of equal high halves into buffer 0, and the complete sort
        // (also ending in buffer 0) only where a run is too long for it
        for (int j = 0; j < 4; ++j) PR_CHECK(pass(L, 32 + 8 * j, j == 0, false, (j + 1) & 1, j & 1, true));
        hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, st, (uint32_t *)flag, (int64_t)1);
        PR_LAUNCHED();
        // ranks through the staging buffer (vals[1], free once the fix-up
        // has read it) where every segment fits the packing, the fix-up
        // then writing the permutation in order (into vals[0] unless asked
        // for) instead of the ranks; the complete sort behind it keeps
        // storing the ranks itself
        uint32_t *perm_fix = perm ? perm : (staged_ranks ? vals[0] : nullptr);
        if (payload)
            hipLaunchKernelGGL((rs_fixup<VAR, true>), grid, dim3(RS_THREADS), 0, st, (const uint64_t *)keys[1],
                               (const uint32_t *)vals[1], (uint64_t *)keys[0], L, staged_ranks ? nullptr : rank,
                               perm_fix, xs, flag);
        else
            hipLaunchKernelGGL((rs_fixup<VAR, false>), grid, dim3(RS_THREADS), 0, st, (const uint64_t *)keys[1],
                               (const uint32_t *)nullptr, (uint64_t *)keys[0], L, rank, perm, xs, flag);
        PR_LAUNCHED();
        if (staged_ranks) PR_CHECK(stage_ranks(perm_fix, vals[1]));
        SortLayout LG = L;
        LG.guard = flag;
        for (int j = 0; j < P; ++j) PR_CHECK(pass(LG, 8 * j, j == 0, j == P - 1, j & 1, (j + 1) & 1, false));
    } else {
        // the last pass reads vals[0] and writes the permutation into vals[1]
        // (unless asked for); vals[0] then stages the ranks
        if (staged_ranks) {
            rank_last = nullptr;
            perm_last = perm ? perm : vals[1];
        }
        for (int j = 0; j < P; ++j) PR_CHECK(pass(L, 8 * j, j == 0, j == P - 1, (j + 1) & 1, j & 1, true));
        if (staged_ranks) {
            hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, st, (uint32_t *)flag, (int64_t)1);
            PR_LAUNCHED();
            PR_CHECK(stage_ranks(perm_last, vals[0]));
        }
    }
    const K *sorted = keys[sorted_buffer<K>()];
    hipLaunchKernelGGL((rs_knots<K, VAR>), dim3(L.nseg), dim3(128), 0, st, sorted, L, nq, q);
    PR_LAUNCHED();
    if (mom) {
        hipLaunchKernelGGL((rs_moments<VAR>), dim3(L.nseg), dim3(64), 0, st, (const double *)mom_part, L, mom);
        PR_LAUNCHED();
    }
    return PR_OK;
}

int restrict_quantiles(const void *x, int precision, int64_t n, int k, int nq, const pr_grid *hg, double *q,
                       uint32_t *rank, uint32_t *perm, double *xs, double *mom, uint32_t *hist, void *ws,
                       hipStream_t st) {
    SortLayout L{n, (int)sort_tiles(n), k, nullptr, nullptr};
    const int64_t tiles = (int64_t)L.nblk * k;
    if (precision == PR_F64)
        return sort_impl<uint64_t, false>(x, L, n * k, tiles, nq, hg, q, rank, perm, xs, mom, hist, ws, st);
    return sort_impl<uint32_t, false>(x, L, n * k, tiles, nq, hg, q, rank, perm, xs, mom, hist, ws, st);
}

int restrict_knots_guarded(const void *x, int precision, int64_t n, int k, int nq, double *q, void *ws,
                           const int *guard, hipStream_t st) {
    SortLayout L{n, (int)sort_tiles(n), k, nullptr, nullptr, guard};
    const int64_t tiles = (int64_t)L.nblk * k;
    if (precision == PR_F64)
        return sort_impl<uint64_t, false>(x, L, n * k, tiles, nq, nullptr, q, nullptr, nullptr, nullptr, nullptr,
                                          nullptr, ws, st);
    return sort_impl<uint32_t, false>(x, L, n * k, tiles, nq, nullptr, q, nullptr, nullptr, nullptr, nullptr,
                                      nullptr, ws, st);
}

int restrict_segments(const void *x, int precision, const SortLayout &L, int64_t total_keys, int64_t total_tiles,
                      int nq, double *q, uint32_t *rank, void *ws, hipStream_t st) {
    if (precision == PR_F64)
        return sort_impl<uint64_t, true>(x, L, total_keys, total_tiles, nq, nullptr, q, rank, nullptr, nullptr,
                                         nullptr, nullptr, ws, st);
    return sort_impl<uint32_t, true>(x, L, total_keys, total_tiles, nq, nullptr, q, rank, nullptr, nullptr, nullptr,
                                     nullptr, ws, st);
}


template <typename K, bool VAR>
static int launch_matched_knots(const MkArgs &A, unsigned ngroups_or_x, int nseg, hipStream_t st) {
    const size_t lds = (size_t)(A.nq + 1) * sizeof(double);
    hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, st, (uint32_t *)A.flag, (int64_t)1);
    PR_LAUNCHED();
    if (A.segflag) {
        hipLaunchKernelGGL(zero_u32, dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, st, (uint32_t *)A.segflag,
                           (int64_t)nseg);
        PR_LAUNCHED();
    }
    const dim3 eg = VAR ? dim3(ngroups_or_x) : dim3(ngroups_or_x, (unsigned)nseg);
    hipLaunchKernelGGL((mk_extremes<K, VAR>), eg, dim3(256), lds, st, A);
    PR_LAUNCHED();
    hipLaunchKernelGGL((mk_scan<K, VAR>), dim3((unsigned)nseg), dim3(256), 0, st, A);
    PR_LAUNCHED();
    hipLaunchKernelGGL((mk_knots<K, VAR>), dim3((unsigned)((A.nq + 1 + 3) / 4), (unsigned)nseg), dim3(256), lds, st,
                       A);
    PR_LAUNCHED();
    return PR_OK;
}

// The workspace as sort_impl lays it out: two key buffers of kb bytes, the
// sorted keys in the one the last pass wrote; the other is free scratch.
template <typename K>
static void key_buffers(const void *ws, size_t kb, const void **sorted, void **scratch) {
    char *p = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    constexpr int last = sorted_buffer<K>();
    *sorted = p + last * kb;
    *scratch = p + (1 - last) * kb;
}

template <typename K>
static int matched_knots_impl(const void *ws, int64_t n, int k, int nq, const double *qt, int64_t qts,
                              const double *qp, int64_t qps, double *q, int *flag, hipStream_t st) {
    const size_t kb = align256((size_t)n * k * sizeof(K));
    const int64_t nch = (n + 63) / 64, ngr = (nch + MK_GROUP - 1) / MK_GROUP;
    if ((size_t)2 * (nch + ngr) * k * sizeof(K) > kb) return PR_E_UNSUPPORTED;
    const void *sorted;
    void *scratch;
    key_buffers<K>(ws, kb, &sorted, &scratch);
    K *pre = (K *)scratch, *suf = pre + nch * k, *gx = suf + nch * k, *gn = gx + ngr * k;
    const MkArgs A{sorted, n, nch, ngr, qt, qp, qts, qps, q, nullptr, nullptr, pre, suf, gx, gn, nq, flag, nullptr};
    return launch_matched_knots<K, false>(A, (unsigned)ngr, k, st);
}

int matched_knots_segments(const void *ws, int64_t total_keys, int nseg, const MkSeg *segs, const int *group_seg,
                           int64_t total_chunks, int64_t total_groups, int nq, const double *qt, const double *qp,
                           double *q, int *flag, int *segflag, hipStream_t st) {
    const size_t kb = align256((size_t)total_keys * sizeof(uint64_t));
    if ((size_t)2 * (total_chunks + total_groups) * sizeof(uint64_t) > kb) return PR_E_UNSUPPORTED;
    const void *sorted;
    void *scratch;
    key_buffers<uint64_t>(ws, kb, &sorted, &scratch);
    uint64_t *pre = (uint64_t *)scratch, *suf = pre + total_chunks, *gx = suf + total_chunks,
             *gn = gx + total_groups;
    const MkArgs A{sorted, 0, 0, 0, qt, qp, 0, 0, q, segs, group_seg, pre, suf, gx, gn, nq, flag, segflag};
    return launch_matched_knots<uint64_t, true>(A, (unsigned)total_groups, nseg, st);
}

int matched_knots(const void *ws, int precision, int64_t n, int k, int nq, const double *qt, int64_t qt_stride,
                  const double *qp, int64_t qp_stride, double *q, int *flag, hipStream_t st) {
    if (precision == PR_F64)
        return matched_knots_impl<uint64_t>(ws, n, k, nq, qt, qt_stride, qp, qp_stride, q, flag, st);
    return matched_knots_impl<uint32_t>(ws, n, k, nq, qt, qt_stride, qp, qp_stride, q, flag, st);
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

// ---------------------------------------------------------------------------
// Restriction without allocation: the workspace is a file-scope device array
// of PR_STATIC_SCRATCH_BYTES (one copy per GPU, held until the process ends).
// Host code never passes the array's name to a kernel: its device address on
// the current GPU is taken once per device with hipGetSymbolAddress and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[PR_STATIC_SCRATCH_BYTES];

namespace pr {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_on_current_device(void **out) {
    int dev = 0;
    PR_HIP(hipGetDevice(&dev));
    PR_REQUIRE(dev >= 0 && dev < kMaxDevices, "device %d outside the %d devices served", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            set_error("hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
            return PR_E_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PR_OK;
}
}  // namespace
}  // namespace pr

extern "C" int pr_restrict_quantiles_static(const void *x, int precision, int64_t n, int k, int n_q,
                                            const pr_grid *hist_grid, double *q, uint32_t *rank, uint32_t *perm,
                                            double *x_sorted, double *moments, uint32_t *hist, void *stream) {
    clear_error();
    PR_REQUIRE(valid_precision(precision), "precision must be 64 or 32");
    PR_REQUIRE(n >= 1 && n <= 0xFFFFFFFFll, "n must be in [1, 2^32)");
    PR_REQUIRE(k >= 1 && k <= 65535, "k must be in [1, 65535]");
    PR_REQUIRE(n_q >= 1 && n_q <= 1 << 20, "n_q must be in [1, 2^20]");
    PR_REQUIRE(x != nullptr && q != nullptr, "x and q must be non-NULL");
    if (hist) {
        PR_REQUIRE(hist_grid != nullptr, "hist requires hist_grid");
        PR_REQUIRE(hist_grid->n_cells >= 1 && hist_grid->n_cells <= 8192 && hist_grid->x_lo < hist_grid->x_hi,
                   "hist_grid must have 1..8192 cells and x_lo < x_hi");
    }
    const size_t need = restrict_ws(n, k, precision);
    if (need > (size_t)PR_STATIC_SCRATCH_BYTES) {
        set_error("n * k = %lld keys need %zu bytes of scratch; the static scratch holds %zu",
                  (long long)n * k, need, (size_t)PR_STATIC_SCRATCH_BYTES);
        return PR_E_NOMEM;
    }
    void *ws = nullptr;
    PR_CHECK(scratch_on_current_device(&ws));
    return restrict_quantiles(x, precision, n, k, n_q, hist_grid, q, rank, perm, x_sorted, moments, hist, ws,
                              as_stream(stream));
}

extern "C" int pr_match_knots(const double *q_target, const double *q_prior, int64_t n, int k, int n_q,
                              int precision, void *ws, size_t ws_bytes, double *q_out, int *flag, void *stream) {
    clear_error();
    PR_REQUIRE(valid_precision(precision), "precision must be 64 or 32");
    PR_REQUIRE(n >= 1 && n <= 0xFFFFFFFFll, "n must be in [1, 2^32)");
    PR_REQUIRE(k >= 1 && k <= 65535, "k must be in [1, 65535]");
    PR_REQUIRE(n_q >= 1 && n_q <= 8191, "n_q must be in [1, 8191]");
    PR_REQUIRE(q_target && q_prior && ws && q_out && flag, "pointers must be non-NULL");
    if (ws_bytes < restrict_ws(n, k, precision)) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, restrict_ws(n, k, precision));
        return PR_E_NOMEM;
    }
    const int rc = matched_knots(ws, precision, n, k, n_q, q_target, n_q + 1, q_prior, n_q + 1, q_out, flag,
                                 as_stream(stream));
    if (rc == PR_E_UNSUPPORTED) set_error("n = %lld is too small for the workspace to hold the chunk extremes",
                                          (long long)n);
    return rc;
}
