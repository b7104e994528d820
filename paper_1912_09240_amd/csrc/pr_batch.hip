// Batched micro-macro parareal: many independent instances of the slow-fast
// SDE (each with its own eps, lambda, particle count P_i, slice count N_i and
// fine step), iterated together.  One iteration is a fixed sequence of
// launches over all instances:
//   fine     one persistent launch: every workgroup takes (instance, slice,
//            particle tile) units from a queue sorted by decreasing cost
//            (longest-processing-time order), until the queue is empty;
//   restrict one segmented sort over all (instance, slice) ensembles of
//            unequal lengths (ranks and knots of the fine results);
//   coarse   the coarse propagator of every (instance, slice) from the
//            previous states, in parallel;
//   chain    one workgroup per instance runs that instance's serial chain
//            (coarse step, quantile iterator, monotone repair) over its slices;
//   match    all (instance, slice) ensembles matched in one launch;
//   knots    one segmented sort of the new states (knots only).
// The sequence can be captured once in a hipGraph per ping-pong parity and
// replayed.  The same handle can also run every phase instance by instance
// with the same kernels (the launch pattern of running the instances one
// after the other); the states are bitwise identical in all modes.
//
// An autotuner times the fine kernel's block size and particles per thread
// on the heaviest units of the batch and keeps the fastest (cached per
// device for the process).
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "pr_coarse_dev.hpp"
#include "pr_fine_dev.hpp"
#include "pr_internal.hpp"

namespace pr {

int build_expm(const std::vector<double> &lo, const std::vector<double> &di, const std::vector<double> &up, int n,
               double tau, double *out, double *w1, double *w2, double *w3, hipStream_t st);
int make_generator(const pr_sde *sde, const pr_grid *grid, std::vector<double> &lo, std::vector<double> &di,
                   std::vector<double> &up, hipStream_t st);

struct InstDev {
    EmCoef<double> c;
    int64_t S;      // fine steps of the instance
    int64_t n;      // particles
    int64_t xoff;   // element offset of time 0 in the state-shaped arrays
    int K;          // slices
    int qrow0;      // knot row of time 0
    uint32_t inst;  // Philox instance word
    int pad;
};

struct Unit {  // fine work unit
    int inst, slice;
    uint32_t p0, np;
};

struct CoarseUnit {  // one (instance, slice) of the coarse propagator
    int in_row, out_row, e_id, pad;
};

struct MatchSeg {
    int64_t base, n;  // state-shaped offset of the ensemble, its length
    int qt_row, qp_row;
    int64_t tile0;
};

struct ChainInst {
    int qrow0, K, u0, pad;  // knot row of time 0, slices, first coarse unit
};

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------
__global__ void zero_counter(unsigned *c) { *c = 0u; }

template <int PPT>
__global__ void __launch_bounds__(256) fine_batch_kernel(const Unit *__restrict__ units, int n_units,
                                                         unsigned *__restrict__ counter,
                                                         const InstDev *__restrict__ insts,
                                                         const double *xin, const double *yin, double *xout,
                                                         double *yout, Key key) {
    __shared__ int u_sh;
    __shared__ NoiseTab tab;
    load_noise_tab(tab);
    const double a1[1] = {1.0};
    for (;;) {
        if (threadIdx.x == 0) u_sh = (int)atomicAdd(counter, 1u);
        __syncthreads();
        // the unit is the block's: in scalar registers, so are its instance's
        // coefficients and the step range
        const int u = __builtin_amdgcn_readfirstlane(u_sh);
        __syncthreads();
        if (u >= n_units) break;  // every wave reaches this once the queue is empty
        const Unit U = units[u];
        const InstDev I = insts[U.inst];
        const int64_t m0 = uniform_i64(slice_begin(I.S, I.K, U.slice));
        const int64_t m1 = uniform_i64(slice_begin(I.S, I.K, U.slice + 1));
        const int64_t src = I.xoff + (int64_t)U.slice * I.n, dst = src + I.n;
        double xv[PPT], yv[PPT][1];
        bool live[PPT];
        uint32_t pp[PPT];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const uint32_t off = threadIdx.x + (uint32_t)q * blockDim.x;
            live[q] = off < U.np;
            pp[q] = U.p0 + (live[q] ? off : 0u);
            xv[q] = xin[src + pp[q]];
            yv[q][0] = yin[src + pp[q]];
        }
        // 32-bit step counter (the generator's counter word is 32 bits wide)
        const uint32_t mb = (uint32_t)m0, steps = (uint32_t)(m1 - m0);
#pragma unroll 2
        for (uint32_t i = 0; i < steps; ++i) {
#pragma unroll
            for (int q = 0; q < PPT; ++q) em_step<1, double>(xv[q], yv[q], a1, I.c, tab, key, I.inst, mb + i, pp[q]);
        }
        for (int q = 0; q < PPT; ++q)
            if (live[q]) {
                xout[dst + pp[q]] = xv[q];
                yout[dst + pp[q]] = yv[q][0];
            }
    }
}

// Coarse propagator over a list of (instance, slice) units: knots -> masses,
// masses -> E masses, masses -> knots.
__global__ void __launch_bounds__(256) k2m_units(const double *__restrict__ q, const CoarseUnit *__restrict__ cu,
                                                 double *__restrict__ rho, GridDev g) {
#pragma clang fp contract(off)
    extern __shared__ double sh[];
    double *qs = sh;
    double *c = sh + g.nq + 1;
    const CoarseUnit U = cu[blockIdx.x];
    for (int j = threadIdx.x; j <= g.nq; j += blockDim.x) qs[j] = q[(int64_t)U.in_row * (g.nq + 1) + j];
    __syncthreads();
    for (int i = 1 + threadIdx.x; i < g.cells; i += blockDim.x) c[i] = cdf_knots(qs, g.nq, edge_at(g, i));
    __syncthreads();
    double *r = rho + (int64_t)blockIdx.x * g.cells;
    for (int i = threadIdx.x; i < g.cells; i += blockDim.x)
        r[i] = (i == 0) ? c[1] : (i == g.cells - 1) ? 1.0 - c[g.cells - 1] : c[i + 1] - c[i];
}

// E rho for 4 rows of one unit per block, one wave per row.
__device__ __forceinline__ double row_dot(const double *row, const double *v, int n, int lane) {
    double acc = lane_row_dot(row, v, n, lane);
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    return acc;
}

__global__ void __launch_bounds__(256) apply_units(const double *__restrict__ E, const CoarseUnit *__restrict__ cu,
                                                   const double *__restrict__ rin, double *__restrict__ rout, int n) {
    extern __shared__ double rv[];
    const int u = blockIdx.y;
    const double *Es = E + (int64_t)cu[u].e_id * n * n;
    for (int j = threadIdx.x; j < n; j += blockDim.x) rv[j] = rin[(int64_t)u * n + j];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + wave;
    if (r >= n) return;
    const double acc = row_dot(Es + (int64_t)r * n, rv, n, lane);
    if (lane == 0) rout[(int64_t)u * n + r] = acc > 0.0 ? acc : 0.0;
}

__global__ void __launch_bounds__(256) m2k_units(const double *__restrict__ rho, const CoarseUnit *__restrict__ cu,
                                                 double *__restrict__ q, GridDev g) {
    extern __shared__ double sh[];
    double *r = sh;
    double *C = sh + g.cells;
    for (int i = threadIdx.x; i < g.cells; i += blockDim.x) r[i] = rho[(int64_t)blockIdx.x * g.cells + i];
    __syncthreads();
    masses_to_knots_block(r, C, g, q + (int64_t)cu[blockIdx.x].out_row * (g.nq + 1));
}

// Serial chain of one instance per block: q_{k+1}^{n+1} = J(C_n(q_{k+1}^n),
// q_f^{n+1}, q_c^{*,n+1}); without qf it is the plain coarse pass of the
// zeroth iteration, q^{n+1} = C_n(q^n).  qn row 0 is copied from q.  A block
// of CHAIN_THREADS: the product E rho of a link is spread over all its waves,
// each taking CHAIN_ROWS rows at a time with their loads in flight together,
// every row summed in the order of the single-instance coarse step.
constexpr int CHAIN_THREADS = 1024;
constexpr int CHAIN_ROWS = 4;

__global__ void __launch_bounds__(CHAIN_THREADS) chain_kernel(const ChainInst *__restrict__ ci, int inst0,
                                                    const CoarseUnit *__restrict__ cu, const double *__restrict__ E,
                                                    const double *__restrict__ q, const double *__restrict__ qf,
                                                    const double *__restrict__ qcs, double *__restrict__ qn,
                                                    GridDev g) {
#pragma clang fp contract(off)
    extern __shared__ double sh[];
    const int Q1 = g.nq + 1;
    double *qc = sh;               // Q1: current knots
    double *c = qc + Q1;           // cells + 1
    double *rho = c + g.cells + 1;  // cells
    double *rho2 = rho + g.cells;   // cells
    double *C = rho2 + g.cells;     // cells + 1
    double *S = C + g.cells + 1;    // Q1
    int *SC = (int *)(S + Q1);      // Q1
    int *vio = SC + Q1;             // Q1
    const ChainInst I = ci[inst0 + blockIdx.x];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int j = threadIdx.x; j < Q1; j += blockDim.x) {
        const double v = q[(int64_t)I.qrow0 * Q1 + j];
        qc[j] = v;
        qn[(int64_t)I.qrow0 * Q1 + j] = v;
    }
    __syncthreads();
    for (int s = 0; s < I.K; ++s) {
        const CoarseUnit U = cu[I.u0 + s];
        for (int i = 1 + threadIdx.x; i < g.cells; i += blockDim.x) c[i] = cdf_knots(qc, g.nq, edge_at(g, i));
        __syncthreads();
        for (int i = threadIdx.x; i < g.cells; i += blockDim.x)
            rho[i] = (i == 0) ? c[1] : (i == g.cells - 1) ? 1.0 - c[g.cells - 1] : c[i + 1] - c[i];
        __syncthreads();
        const double *Es = E + (int64_t)U.e_id * g.cells * g.cells;
        const int nw = (int)(blockDim.x >> 6);
        for (int r0 = wave; r0 < g.cells; r0 += nw * CHAIN_ROWS) {
            const double *rows[CHAIN_ROWS];
            double acc[CHAIN_ROWS];
#pragma unroll
            for (int k = 0; k < CHAIN_ROWS; ++k) {
                const int r = r0 + k * nw;
                rows[k] = Es + (int64_t)(r < g.cells ? r : r0) * g.cells;
            }
            lane_rows_dot<CHAIN_ROWS, 4>(rows, rho, g.cells, lane, acc);
#pragma unroll
            for (int k = 0; k < CHAIN_ROWS; ++k) {
                double a = acc[k];
                for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off);
                const int r = r0 + k * nw;
                if (lane == 0 && r < g.cells) rho2[r] = a > 0.0 ? a : 0.0;
            }
        }
        __syncthreads();
        masses_to_knots_block(rho2, C, g, qc);
        __syncthreads();
        const int64_t orow = (int64_t)U.out_row * Q1;
        if (qf) {
            for (int j = threadIdx.x; j < Q1; j += blockDim.x) qc[j] = qf[orow + j] + (qc[j] - qcs[orow + j]);
            __syncthreads();
            pava_block(qc, Q1, S, SC, vio);
        }
        for (int j = threadIdx.x; j < Q1; j += blockDim.x) qn[orow + j] = qc[j];
        __syncthreads();
    }
}

// Matching over a list of ensembles (tiles of MB_TILE particles).
constexpr int MB_TILE = 1024;

__global__ void __launch_bounds__(256) match_batch_kernel(const MatchSeg *__restrict__ segs,
                                                          const int *__restrict__ tile_seg, int tile_first,
                                                          const double *__restrict__ qt, const double *__restrict__ qp,
                                                          int nq, const uint32_t *__restrict__ rank,
                                                          double *__restrict__ x) {
#pragma clang fp contract(off)
    extern __shared__ double dk[];
    const int t = tile_first + blockIdx.x;
    const MatchSeg M = segs[tile_seg[t]];
    for (int j = threadIdx.x; j <= nq; j += blockDim.x)
        dk[j] = qt[(int64_t)M.qt_row * (nq + 1) + j] - qp[(int64_t)M.qp_row * (nq + 1) + j];
    __syncthreads();
    const double nd = (double)M.n, Q = (double)nq;
    const int64_t p0 = (int64_t)(t - M.tile0) * MB_TILE;
    for (int k = threadIdx.x; k < MB_TILE; k += blockDim.x) {
        const int64_t p = p0 + k;
        if (p >= M.n) break;
        x[M.base + p] = matched_value<double>(x[M.base + p], rank[M.base + p], dk, nd, Q);
    }
}

// After the zeroth iteration: the time-0 state of every instance into the
// other ping-pong buffer, and the fast variables of time 0 into every later
// time point of buffer 0 (matching moves the slow variable only).  One
// launch for the whole batch: blockIdx.y is the instance.
__global__ void spread_time0(const InstDev *__restrict__ insts, double *__restrict__ x0, double *__restrict__ y0,
                             double *__restrict__ x1, double *__restrict__ y1) {
    const InstDev I = insts[blockIdx.y];
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < I.n; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = I.xoff + p;
        const double xv = x0[o], yv = y0[o];
        x1[o] = xv;
        y1[o] = yv;
        for (int t = 1; t <= I.K; ++t) y0[o + (int64_t)t * I.n] = yv;
    }
}

__global__ void copy_f64(const double *__restrict__ a, double *__restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

__global__ void draw_instances_kernel(double *out, int count, Key key) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const Block b = noise_block(key, (uint32_t)i, 3u, 0u, 0u, 0u);
    const double u0 = ((double)b.w0 + 0.5) * 0x1p-32, u1 = ((double)b.w1 + 0.5) * 0x1p-32;
    const double u2 = ((double)b.w2 + 0.5) * 0x1p-32, u3 = ((double)b.w3 + 0.5) * 0x1p-32;
    out[4 * i + 0] = pow(10.0, -3.0 + 2.0 * u0);
    out[4 * i + 1] = 0.5 + 1.5 * u1;
    out[4 * i + 2] = (double)(12 + (int)floor(7.0 * u2));
    out[4 * i + 3] = (double)(8 + (int)floor(57.0 * u3));
}

// ---------------------------------------------------------------------------
// Handle.
// ---------------------------------------------------------------------------
struct Tuned {
    int block = 256, ppt = 2;
};

static std::mutex g_tune_mu;
static std::map<std::string, Tuned> g_tune_cache;

struct Batch {
    int B = 0, Q = 0, flags = 0;
    uint64_t seed = 0;
    pr_grid grid{};
    GridDev g{};
    std::vector<pr_sde> sde;
    std::vector<pr_schedule> sch;
    std::vector<int64_t> n;
    std::vector<uint32_t> inst_id;
    std::vector<InstDev> inst_h;
    std::vector<int64_t> xoff;   // state-shaped offsets
    std::vector<int> qrow0;      // knot row of time 0
    int64_t total_x = 0;          // state-shaped elements
    int total_rows = 0;           // knot rows
    int total_slices = 0;
    // device
    InstDev *inst = nullptr;
    double *x[2] = {nullptr, nullptr}, *y[2] = {nullptr, nullptr};
    double *q = nullptr, *qn = nullptr, *qR = nullptr, *qf = nullptr, *qcs = nullptr;
    uint32_t *rank = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    double *E = nullptr;
    int n_e = 0;
    CoarseUnit *cu = nullptr;           // [total_slices]: in_row = time n, out_row = time n+1
    ChainInst *chain = nullptr;          // [B]
    std::vector<ChainInst> chain_h;
    double *rho_a = nullptr, *rho_b = nullptr;
    // fine work queue
    Unit *units = nullptr;
    int n_units = 0;
    std::vector<Unit> units_h;
    unsigned *counter = nullptr;
    int persist_blocks = 0;
    Tuned tuned;
    // sorts: fine results (t = 1..K_i of every instance) and time 0
    SortSeg *seg_f = nullptr;
    int *tile_f = nullptr;
    int64_t tiles_f = 0, keys_f = 0, seg_max_n = 0;
    std::vector<SortSeg> seg_f_h;
    // the same ensembles in two layouts for the sort of every iteration:
    // those the splitter sort takes, and the rest (radix passes)
    struct Part {
        SortSeg *seg = nullptr;
        int *tile = nullptr;
        int nseg = 0;
        int64_t tiles = 0, min_n = 0, max_n = 0;
    } part[2];
    bool split_sort = true;  // the two layouts above (else one radix sort of all ensembles)
    // matching
    MatchSeg *mseg = nullptr;
    int *mtile = nullptr;
    int n_mtiles = 0;
    std::vector<int> mtile_first;  // per instance
    std::vector<int> mtile_count;
    // knots of the new states from the fine results' sort (chunk and group
    // extremes of every fine-result ensemble), a guarded sort where that fails
    MkSeg *mk_seg = nullptr;
    int *mk_gseg = nullptr;
    int64_t mk_chunks = 0, mk_groups = 0;
    int *flag = nullptr;
    int *flag_host = nullptr;  // pinned copy of flag
    int *segflag = nullptr;    // one flag per fine-result ensemble
    int *segflag_host = nullptr;
    // the segment and tile tables of the ensembles whose knots need the sort
    // (pinned host staging, device copies)
    SortSeg *seg_sub_h = nullptr, *seg_sub = nullptr;
    int *tile_sub_h = nullptr, *tile_sub = nullptr;
    bool mk_ok = true;           // the matched-knot kernels serve this batch
    int knot_sorts = 0;          // batched iterations whose new knots needed the sort
    int64_t knot_sort_segs = 0;  // ensembles sorted by them
    int cur = 0, k = 0;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    double last_ms = 0.0;
};

static void batch_free(Batch *b) {
    if (!b) return;
    void *ptrs[] = {b->inst, b->x[0], b->x[1], b->y[0], b->y[1], b->q, b->qn, b->qR, b->qf, b->qcs, b->rank,
                    b->ws, b->E, b->cu, b->chain, b->rho_a, b->units, b->counter, b->seg_f, b->tile_f, b->mseg,
                    b->mtile, b->mk_seg, b->mk_gseg, b->flag, b->segflag, b->seg_sub, b->tile_sub,
                    b->part[0].seg, b->part[0].tile, b->part[1].seg, b->part[1].tile};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto &gx : b->graph)
        if (gx) (void)hipGraphExecDestroy(gx);
    for (auto &e : b->ev)
        if (e) (void)hipEventDestroy(e);
    void *pinned[] = {b->flag_host, b->segflag_host, b->seg_sub_h, b->tile_sub_h};
    for (void *p : pinned)
        if (p) (void)hipHostFree(p);
    delete b;
}

#define PB_ALLOC(ptr, bytes)                                                        \
    do {                                                                            \
        if (hipMalloc((void **)&(ptr), (bytes)) != hipSuccess) {                    \
            set_error("device allocation of %zu bytes failed", (size_t)(bytes));    \
            return PR_E_NOMEM;                                                      \
        }                                                                           \
    } while (0)

template <typename T>
static int upload(T *&dev, const std::vector<T> &h, hipStream_t st) {
    PB_ALLOC(dev, sizeof(T) * std::max<size_t>(1, h.size()));
    if (!h.empty()) PR_HIP(hipMemcpyAsync(dev, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, st));
    return PR_OK;
}

static size_t lds_chain(const GridDev &g) {
    return sizeof(double) * (2 * (g.nq + 1) + 4 * g.cells + 2) + 2 * sizeof(int) * (g.nq + 1);
}

// Fine units of a given tile size, in decreasing cost.
static void build_units(Batch *b, int tile) {
    b->units_h.clear();
    for (int i = 0; i < b->B; ++i) {
        const int K = b->sch[i].n_slices;
        for (int s = 0; s < K; ++s)
            for (int64_t p0 = 0; p0 < b->n[i]; p0 += tile)
                b->units_h.push_back(Unit{i, s, (uint32_t)p0, (uint32_t)std::min<int64_t>(tile, b->n[i] - p0)});
    }
    auto cost = [&](const Unit &u) {
        const pr_schedule &S = b->sch[u.inst];
        const int64_t L = slice_begin(S.total_steps, S.n_slices, u.slice + 1) - slice_begin(S.total_steps, S.n_slices, u.slice);
        return (double)L * u.np;
    };
    std::stable_sort(b->units_h.begin(), b->units_h.end(),
                     [&](const Unit &a, const Unit &c) { return cost(a) > cost(c); });
    b->n_units = (int)b->units_h.size();
}

// Resident workgroups of the persistent fine kernel (queried outside any
// stream capture).
template <int PPT, int BS>
static int fine_batch_slots(int &slots) {
    int per_cu = 0, dev = 0, cus = 0;
    PR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fine_batch_kernel<PPT>, BS, 0));
    PR_HIP(hipGetDevice(&dev));
    PR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    slots = std::max(1, per_cu * cus);
    return PR_OK;
}

static int fine_slots(const Tuned &t, int &slots) {
    if (t.block == 256 && t.ppt == 1) return fine_batch_slots<1, 256>(slots);
    if (t.block == 256 && t.ppt == 2) return fine_batch_slots<2, 256>(slots);
    if (t.block == 256 && t.ppt == 4) return fine_batch_slots<4, 256>(slots);
    if (t.block == 128 && t.ppt == 1) return fine_batch_slots<1, 128>(slots);
    if (t.block == 128 && t.ppt == 2) return fine_batch_slots<2, 128>(slots);
    return fine_batch_slots<4, 128>(slots);
}

template <int PPT, int BS>
static int launch_fine_batch(Batch *b, int n_units, int c, int nx, hipStream_t st) {
    hipLaunchKernelGGL(zero_counter, dim3(1), dim3(1), 0, st, b->counter);
    PR_LAUNCHED();
    const int grid = std::max(1, std::min(n_units, b->persist_blocks));
    hipLaunchKernelGGL((fine_batch_kernel<PPT>), dim3(grid), dim3(BS), 0, st, (const Unit *)b->units, n_units,
                       b->counter, (const InstDev *)b->inst, (const double *)b->x[c], (const double *)b->y[c],
                       b->x[nx], b->y[nx], make_key(b->seed));
    PR_LAUNCHED();
    return PR_OK;
}

static int fine_batch(Batch *b, int n_units, int c, int nx, hipStream_t st) {
    const Tuned &t = b->tuned;
    if (t.block == 256 && t.ppt == 1) return launch_fine_batch<1, 256>(b, n_units, c, nx, st);
    if (t.block == 256 && t.ppt == 2) return launch_fine_batch<2, 256>(b, n_units, c, nx, st);
    if (t.block == 256 && t.ppt == 4) return launch_fine_batch<4, 256>(b, n_units, c, nx, st);
    if (t.block == 128 && t.ppt == 1) return launch_fine_batch<1, 128>(b, n_units, c, nx, st);
    if (t.block == 128 && t.ppt == 2) return launch_fine_batch<2, 128>(b, n_units, c, nx, st);
    return launch_fine_batch<4, 128>(b, n_units, c, nx, st);
}

// Times the fine kernel shapes on the heaviest units of the batch.
static int autotune(Batch *b, hipStream_t st) {
    int dev = 0;
    PR_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    PR_HIP(hipGetDeviceProperties(&prop, dev));
    const std::string keyname = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "/d1f64";
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(keyname);
        if (it != g_tune_cache.end()) {
            b->tuned = it->second;
            return PR_OK;
        }
    }
    const Tuned cands[] = {{256, 1}, {256, 2}, {256, 4}, {128, 1}, {128, 2}, {128, 4}};
    hipEvent_t e0, e1;
    PR_HIP(hipEventCreate(&e0));
    PR_HIP(hipEventCreate(&e1));
    double best = 1e300;
    Tuned pick = b->tuned;
    for (const Tuned &cnd : cands) {
        b->tuned = cnd;
        PR_CHECK(fine_slots(cnd, b->persist_blocks));
        build_units(b, cnd.block * cnd.ppt);
        PR_CHECK(upload(b->units, b->units_h, st));
        // the heaviest units, about 2e9 particle-steps of work
        int nu = 0;
        double work = 0.0;
        while (nu < b->n_units && work < 2e9) {
            const Unit &u = b->units_h[nu];
            const pr_schedule &S = b->sch[u.inst];
            work += (double)(slice_begin(S.total_steps, S.n_slices, u.slice + 1) -
                             slice_begin(S.total_steps, S.n_slices, u.slice)) * u.np;
            ++nu;
        }
        PR_CHECK(fine_batch(b, nu, b->cur, 1 - b->cur, st));  // warm-up
        PR_HIP(hipEventRecord(e0, st));
        PR_CHECK(fine_batch(b, nu, b->cur, 1 - b->cur, st));
        PR_HIP(hipEventRecord(e1, st));
        PR_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        PR_HIP(hipEventElapsedTime(&ms, e0, e1));
        const double rate = ms / work;
        if (rate < best) {
            best = rate;
            pick = cnd;
        }
        (void)hipFree(b->units);
        b->units = nullptr;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->tuned = pick;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[keyname] = pick;
    return PR_OK;
}

// Restriction of the fine results (buffer nx): knots into qf, ranks; in the
// two layouts (splitter sort for the ensembles it takes, radix passes for the
// rest) or as one segment table by radix passes, as tuned.
static int restrict_fine(Batch *b, int nx, hipStream_t st) {
    if (!b->split_sort) {
        const SortLayout L{0, 0, (int)b->seg_f_h.size(), b->seg_f, b->tile_f, nullptr, b->seg_max_n};
        return restrict_segments(b->x[nx], PR_F64, L, b->total_x, b->tiles_f, b->Q, b->qf, b->rank, b->ws, st);
    }
    for (const Batch::Part &P : b->part) {
        if (P.nseg == 0) continue;
        const SortLayout LP{0, 0, P.nseg, P.seg, P.tile, nullptr, P.max_n, P.min_n};
        PR_CHECK(restrict_segments(b->x[nx], PR_F64, LP, b->total_x, P.tiles, b->Q, b->qf, b->rank, b->ws, st));
    }
    return PR_OK;
}

// Times the two restrictions of the fine results on the batch's own states
// (those of the zeroth iteration, the same shapes) and keeps the faster; both
// give the same bits.  The outputs it writes are rewritten by the first
// iteration.
static int tune_sort(Batch *b, hipStream_t st) {
    if (b->part[0].nseg == 0) {  // no ensemble the splitter sort takes
        b->split_sort = false;
        return PR_OK;
    }
    hipEvent_t e0, e1;
    PR_HIP(hipEventCreate(&e0));
    PR_HIP(hipEventCreate(&e1));
    double ms_of[2] = {0.0, 0.0};
    int rc = PR_OK;
    for (int split = 0; split < 2 && rc == PR_OK; ++split) {
        b->split_sort = split == 1;
        rc = restrict_fine(b, b->cur, st);  // warm-up
        if (rc != PR_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) rc = PR_E_HIP;
        if (rc == PR_OK) rc = restrict_fine(b, b->cur, st);
        if (rc == PR_OK && hipEventRecord(e1, st) != hipSuccess) rc = PR_E_HIP;
        if (rc == PR_OK && hipEventSynchronize(e1) != hipSuccess) rc = PR_E_HIP;
        float ms = 0.f;
        if (rc == PR_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = PR_E_HIP;
        ms_of[split] = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != PR_OK) {
        set_error("timing the restriction of the fine results failed");
        return rc;
    }
    b->split_sort = ms_of[1] <= ms_of[0];
    return PR_OK;
}

// After a batched iteration (buffer nx holds the new states): where the
// matched-knot kernels raised the flag, the knots of the new states come from
// a sort of them.  The host reads the flag once per iteration instead of
// launching the sort guarded by it, whose empty launches cost more than the
// wait.  Only the ensembles whose own flag is raised are sorted: their
// segment entries (state offset, length, knot row) with tiles renumbered
// from 0 make the layout of that sort.
static int sort_new_if_flagged(Batch *b, int nx, hipStream_t st) {
    if (!b->mk_ok) return PR_OK;
    PR_HIP(hipMemcpyAsync(b->flag_host, b->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    PR_HIP(hipStreamSynchronize(st));
    if (*b->flag_host == 0) return PR_OK;
    const int nseg = (int)b->seg_f_h.size();
    PR_HIP(hipMemcpyAsync(b->segflag_host, b->segflag, sizeof(int) * nseg, hipMemcpyDeviceToHost, st));
    PR_HIP(hipStreamSynchronize(st));
    int nsub = 0;
    int64_t tiles = 0, max_n = 0;
    for (int s = 0; s < nseg; ++s) {
        if (!b->segflag_host[s]) continue;
        SortSeg g = b->seg_f_h[s];
        g.tile0 = tiles;
        for (int t = 0; t < g.nblk; ++t) b->tile_sub_h[tiles + t] = nsub;
        b->seg_sub_h[nsub++] = g;
        tiles += g.nblk;
        max_n = std::max(max_n, g.n);
    }
    PR_REQUIRE(nsub > 0 && tiles <= b->tiles_f, "matched-knot flags inconsistent");
    PR_HIP(hipMemcpyAsync(b->seg_sub, b->seg_sub_h, sizeof(SortSeg) * nsub, hipMemcpyHostToDevice, st));
    PR_HIP(hipMemcpyAsync(b->tile_sub, b->tile_sub_h, sizeof(int) * tiles, hipMemcpyHostToDevice, st));
    SortLayout L{0, 0, nsub, b->seg_sub, b->tile_sub, nullptr, max_n};
    PR_CHECK(restrict_segments(b->x[nx], PR_F64, L, b->total_x, tiles, b->Q, b->qR, nullptr, b->ws, st));
    b->knot_sorts += 1;
    b->knot_sort_segs += nsub;
    return PR_OK;
}

// One iteration: mode 0 = batched launches, 1 = instance by instance.
static int iterate_once(Batch *b, int mode, hipStream_t st) {
    const int c = b->cur, nx = 1 - c, Q = b->Q;
    const GridDev &g = b->g;
    if (mode == 0) {
        PR_CHECK(fine_batch(b, b->n_units, c, nx, st));
        SortLayout L{0, 0, (int)b->seg_f_h.size(), b->seg_f, b->tile_f, nullptr, b->seg_max_n};
        PR_CHECK(restrict_fine(b, nx, st));
        const double *cin = (b->flags & PR_REUSE_COARSE) ? b->q : b->qR;
        hipLaunchKernelGGL(k2m_units, dim3(b->total_slices), dim3(256), sizeof(double) * (g.nq + g.cells + 2), st,
                           cin, (const CoarseUnit *)b->cu, b->rho_a, g);
        PR_LAUNCHED();
        hipLaunchKernelGGL(apply_units, dim3((g.cells + 3) / 4, b->total_slices), dim3(256),
                           sizeof(double) * g.cells, st, (const double *)b->E, (const CoarseUnit *)b->cu,
                           (const double *)b->rho_a, b->rho_b, g.cells);
        PR_LAUNCHED();
        hipLaunchKernelGGL(m2k_units, dim3(b->total_slices), dim3(256), sizeof(double) * (2 * g.cells + 1), st,
                           (const double *)b->rho_b, (const CoarseUnit *)b->cu, b->qcs, g);
        PR_LAUNCHED();
        hipLaunchKernelGGL(chain_kernel, dim3(b->B), dim3(CHAIN_THREADS), lds_chain(g), st, (const ChainInst *)b->chain, 0,
                           (const CoarseUnit *)b->cu, (const double *)b->E, (const double *)b->q,
                           (const double *)b->qf, (const double *)b->qcs, b->qn, g);
        PR_LAUNCHED();
        hipLaunchKernelGGL(match_batch_kernel, dim3(b->n_mtiles), dim3(256), sizeof(double) * (Q + 1), st,
                           (const MatchSeg *)b->mseg, (const int *)b->mtile, 0, (const double *)b->qn,
                           (const double *)b->qf, Q, (const uint32_t *)b->rank, b->x[nx]);
        PR_LAUNCHED();
        // knots of the new states: from the fine results' sort; where that
        // cannot isolate every order statistic the device raises the flag and
        // the host sorts the new states after the iteration (sort_new_if_flagged)
        const int mk = matched_knots_segments(b->ws, b->total_x, (int)b->seg_f_h.size(), b->mk_seg, b->mk_gseg,
                                              b->mk_chunks, b->mk_groups, Q, b->qn, b->qf, b->qR, b->flag,
                                              b->segflag, st);
        if (mk != PR_OK && mk != PR_E_UNSUPPORTED) return mk;
        b->mk_ok = mk == PR_OK;
        if (!b->mk_ok)
            PR_CHECK(restrict_segments(b->x[nx], PR_F64, L, b->total_x, b->tiles_f, Q, b->qR, nullptr, b->ws, st));
        hipLaunchKernelGGL(copy_f64, dim3(64), dim3(256), 0, st, (const double *)b->qn, b->q,
                           (int64_t)b->total_rows * (Q + 1));
        PR_LAUNCHED();
    } else {
        for (int i = 0; i < b->B; ++i) {
            const int K = b->sch[i].n_slices;
            const int64_t n = b->n[i], xo = b->xoff[i];
            const int r0 = b->qrow0[i];
            const ChainInst &ci = b->chain_h[i];
            PR_CHECK(fine_propagate(&b->sde[i], &b->sch[i], b->seed, b->inst_id[i], n, 0, K, b->x[c] + xo,
                                    b->y[c] + xo, b->x[nx] + xo + n, b->y[nx] + xo + n, st));
            PR_CHECK(restrict_quantiles(b->x[nx] + xo + n, PR_F64, n, K, Q, nullptr, b->qf + (int64_t)(r0 + 1) * (Q + 1),
                                        b->rank + xo + n, nullptr, nullptr, nullptr, nullptr, b->ws, st));
            const double *cin = (b->flags & PR_REUSE_COARSE) ? b->q : b->qR;
            const CoarseUnit *cu = b->cu + ci.u0;
            hipLaunchKernelGGL(k2m_units, dim3(K), dim3(256), sizeof(double) * (g.nq + g.cells + 2), st, cin, cu,
                               b->rho_a, g);
            PR_LAUNCHED();
            hipLaunchKernelGGL(apply_units, dim3((g.cells + 3) / 4, K), dim3(256), sizeof(double) * g.cells, st,
                               (const double *)b->E, cu, (const double *)b->rho_a, b->rho_b, g.cells);
            PR_LAUNCHED();
            hipLaunchKernelGGL(m2k_units, dim3(K), dim3(256), sizeof(double) * (2 * g.cells + 1), st,
                               (const double *)b->rho_b, cu, b->qcs, g);
            PR_LAUNCHED();
            hipLaunchKernelGGL(chain_kernel, dim3(1), dim3(CHAIN_THREADS), lds_chain(g), st, (const ChainInst *)b->chain, i,
                               (const CoarseUnit *)b->cu, (const double *)b->E, (const double *)b->q,
                               (const double *)b->qf, (const double *)b->qcs, b->qn, g);
            PR_LAUNCHED();
            hipLaunchKernelGGL(match_batch_kernel, dim3(b->mtile_count[i]), dim3(256), sizeof(double) * (Q + 1), st,
                               (const MatchSeg *)b->mseg, (const int *)b->mtile, b->mtile_first[i],
                               (const double *)b->qn, (const double *)b->qf, Q, (const uint32_t *)b->rank, b->x[nx]);
            PR_LAUNCHED();
            double *qr = b->qR + (int64_t)(r0 + 1) * (Q + 1);
            const int mk = matched_knots(b->ws, PR_F64, n, K, Q, b->qn + (int64_t)(r0 + 1) * (Q + 1), Q + 1,
                                         b->qf + (int64_t)(r0 + 1) * (Q + 1), Q + 1, qr, b->flag, st);
            if (mk == PR_OK)
                PR_CHECK(restrict_knots_guarded(b->x[nx] + xo + n, PR_F64, n, K, Q, qr, b->ws, b->flag, st));
            else if (mk == PR_E_UNSUPPORTED)
                PR_CHECK(restrict_quantiles(b->x[nx] + xo + n, PR_F64, n, K, Q, nullptr, qr, nullptr, nullptr,
                                            nullptr, nullptr, nullptr, b->ws, st));
            else
                return mk;
            hipLaunchKernelGGL(copy_f64, dim3(1), dim3(256), 0, st, (const double *)(b->qn + (int64_t)r0 * (Q + 1)),
                               b->q + (int64_t)r0 * (Q + 1), (int64_t)(K + 1) * (Q + 1));
            PR_LAUNCHED();
        }
    }
    return PR_OK;
}

static int batch_create(int B, const pr_sde *sde, const pr_schedule *sch, const int64_t *n, const pr_grid *grid,
                        uint64_t seed, const uint32_t *inst_ids, int flags, hipStream_t st, Batch *b) {
    b->B = B;
    b->Q = grid->n_q;
    b->flags = flags;
    b->seed = seed;
    b->grid = *grid;
    const int I = grid->n_cells;
    const double h = (grid->x_hi - grid->x_lo) / I;
    b->g = GridDev{I, grid->n_q, grid->x_lo, h};
    b->sde.assign(sde, sde + B);
    b->sch.assign(sch, sch + B);
    b->n.assign(n, n + B);
    b->inst_id.resize(B);
    for (int i = 0; i < B; ++i) b->inst_id[i] = inst_ids ? inst_ids[i] : (uint32_t)i;
    // offsets
    b->xoff.resize(B);
    b->qrow0.resize(B);
    int64_t xo = 0;
    int row = 0, slices = 0;
    for (int i = 0; i < B; ++i) {
        b->xoff[i] = xo;
        b->qrow0[i] = row;
        xo += (int64_t)(sch[i].n_slices + 1) * n[i];
        row += sch[i].n_slices + 1;
        slices += sch[i].n_slices;
    }
    b->total_x = xo;
    b->total_rows = row;
    b->total_slices = slices;
    for (int i = 0; i < B; ++i) {
        InstDev d{};
        d.c = make_coef<double>(&sde[i], sch[i].dt);
        d.S = sch[i].total_steps;
        d.n = n[i];
        d.xoff = b->xoff[i];
        d.K = sch[i].n_slices;
        d.qrow0 = b->qrow0[i];
        d.inst = b->inst_id[i];
        b->inst_h.push_back(d);
    }
    PR_CHECK(upload(b->inst, b->inst_h, st));
    const size_t xb = sizeof(double) * (size_t)xo, qb = sizeof(double) * (size_t)row * (b->Q + 1);
    for (int p = 0; p < 2; ++p) {
        PB_ALLOC(b->x[p], xb);
        PB_ALLOC(b->y[p], xb);
    }
    PB_ALLOC(b->q, qb);
    PB_ALLOC(b->qn, qb);
    PB_ALLOC(b->qR, qb);
    PB_ALLOC(b->qf, qb);
    PB_ALLOC(b->qcs, qb);
    PB_ALLOC(b->rank, sizeof(uint32_t) * (size_t)xo);
    PB_ALLOC(b->counter, sizeof(unsigned));
    PB_ALLOC(b->rho_a, sizeof(double) * (size_t)I * slices * 2);
    b->rho_b = b->rho_a + (size_t)I * slices;
    // coarse: one generator per distinct (c3, c1, lambda(1 - abar), beta); E per (generator, slice length)
    std::vector<CoarseUnit> cu;
    std::vector<ChainInst> chain;
    std::vector<std::tuple<double, double, double, double>> gen_keys;
    std::vector<std::vector<double>> G_lo, G_di, G_up;
    struct EReq { int gen; double tau; };
    std::vector<EReq> ereq;
    for (int i = 0; i < B; ++i) {
        if (sde[i].a != nullptr) {
            set_error("batched instances serve a = NULL");
            return PR_E_UNSUPPORTED;
        }
        const auto gk = std::make_tuple(sde[i].c3, sde[i].c1, 0.0, sde[i].beta);  // a = 1: lambda drops out
        int gid = -1;
        for (size_t t = 0; t < gen_keys.size(); ++t)
            if (gen_keys[t] == gk) gid = (int)t;
        if (gid < 0) {
            gid = (int)gen_keys.size();
            gen_keys.push_back(gk);
            std::vector<double> lo, di, up;
            PR_CHECK(make_generator(&sde[i], grid, lo, di, up, st));
            G_lo.push_back(lo);
            G_di.push_back(di);
            G_up.push_back(up);
        }
        chain.push_back(ChainInst{b->qrow0[i], sch[i].n_slices, (int)cu.size(), 0});
        for (int s = 0; s < sch[i].n_slices; ++s) {
            const int64_t L = slice_begin(sch[i].total_steps, sch[i].n_slices, s + 1) -
                              slice_begin(sch[i].total_steps, sch[i].n_slices, s);
            // distinct (generator, tau): tau = L dt of this instance
            const double tau = (double)L * sch[i].dt;
            int eid = -1;
            for (size_t t = 0; t < ereq.size(); ++t)
                if (ereq[t].gen == gid && ereq[t].tau == tau) eid = (int)t;
            if (eid < 0) {
                eid = (int)ereq.size();
                ereq.push_back(EReq{gid, tau});
            }
            cu.push_back(CoarseUnit{b->qrow0[i] + s, b->qrow0[i] + s + 1, eid, 0});
        }
    }
    b->chain_h = chain;
    PR_CHECK(upload(b->cu, cu, st));
    PR_CHECK(upload(b->chain, chain, st));
    b->n_e = (int)ereq.size();
    const int64_t nn = (int64_t)I * I;
    PB_ALLOC(b->E, sizeof(double) * nn * b->n_e);
    {
        double *w = nullptr;
        PB_ALLOC(w, sizeof(double) * nn * 3);
        for (int e = 0; e < b->n_e; ++e) {
            const int s = build_expm(G_lo[ereq[e].gen], G_di[ereq[e].gen], G_up[ereq[e].gen], I, ereq[e].tau,
                                     b->E + nn * e, w, w + nn, w + 2 * nn, st);
            if (s != PR_OK) {
                (void)hipFree(w);
                return s;
            }
        }
        (void)hipFree(w);
    }
    // sort layout of the states t = 1..K_i of every instance
    int64_t tiles = 0, keys = 0;
    std::vector<int> tile_seg;
    for (int i = 0; i < B; ++i)
        for (int s = 0; s < sch[i].n_slices; ++s) {
            SortSeg g{};
            g.base = b->xoff[i] + (int64_t)(s + 1) * n[i];
            g.n = n[i];
            g.tile0 = tiles;
            g.nblk = (int)sort_tiles(n[i]);
            g.qrow = b->qrow0[i] + s + 1;
            for (int t = 0; t < g.nblk; ++t) tile_seg.push_back((int)b->seg_f_h.size());
            b->seg_f_h.push_back(g);
            tiles += g.nblk;
            keys += n[i];
            b->seg_max_n = std::max(b->seg_max_n, (int64_t)n[i]);
        }
    b->tiles_f = tiles;
    b->keys_f = keys;
    PR_CHECK(upload(b->seg_f, b->seg_f_h, st));
    PR_CHECK(upload(b->tile_f, tile_seg, st));
    for (int k = 0; k < 2; ++k) {
        Batch::Part &P = b->part[k];
        std::vector<SortSeg> segs;
        std::vector<int> tl;
        for (const SortSeg &g0 : b->seg_f_h) {
            if (splitter_sorts(g0.n) != (k == 0)) continue;
            SortSeg g = g0;
            g.tile0 = P.tiles;
            for (int t = 0; t < g.nblk; ++t) tl.push_back((int)segs.size());
            segs.push_back(g);
            P.tiles += g.nblk;
            P.min_n = P.min_n == 0 ? g.n : std::min(P.min_n, g.n);
            P.max_n = std::max(P.max_n, g.n);
        }
        P.nseg = (int)segs.size();
        if (P.nseg == 0) continue;
        PR_CHECK(upload(P.seg, segs, st));
        PR_CHECK(upload(P.tile, tl, st));
    }
    {
        std::vector<MkSeg> mk;
        std::vector<int> gseg;
        for (const SortSeg &g : b->seg_f_h) {
            const int64_t nch = (g.n + 63) / 64, ngr = (nch + 63) / 64;
            mk.push_back(MkSeg{g.base, g.n, b->mk_chunks, b->mk_groups, g.qrow, g.qrow, g.qrow, 0});
            for (int64_t t = 0; t < ngr; ++t) gseg.push_back((int)mk.size() - 1);
            b->mk_chunks += nch;
            b->mk_groups += ngr;
        }
        PR_CHECK(upload(b->mk_seg, mk, st));
        PR_CHECK(upload(b->mk_gseg, gseg, st));
        PB_ALLOC(b->flag, sizeof(int));
        PR_HIP(hipHostMalloc((void **)&b->flag_host, sizeof(int), hipHostMallocDefault));
        const size_t nseg = b->seg_f_h.size();
        PB_ALLOC(b->segflag, sizeof(int) * nseg);
        PR_HIP(hipHostMalloc((void **)&b->segflag_host, sizeof(int) * nseg, hipHostMallocDefault));
        PB_ALLOC(b->seg_sub, sizeof(SortSeg) * nseg);
        PR_HIP(hipHostMalloc((void **)&b->seg_sub_h, sizeof(SortSeg) * nseg, hipHostMallocDefault));
        PB_ALLOC(b->tile_sub, sizeof(int) * (size_t)tiles);
        PR_HIP(hipHostMalloc((void **)&b->tile_sub_h, sizeof(int) * (size_t)tiles, hipHostMallocDefault));
    }
    // the sort arrays are indexed like the states (segment bases are state offsets)
    int64_t max_inst_keys = 0, max_inst_tiles = 0;
    int max_k = 1;
    for (int i = 0; i < B; ++i) {
        max_inst_keys = std::max<int64_t>(max_inst_keys, (int64_t)sch[i].n_slices * n[i]);
        max_inst_tiles = std::max<int64_t>(max_inst_tiles, (int64_t)(sch[i].n_slices + 1) * sort_tiles(n[i]));
        max_k = std::max(max_k, sch[i].n_slices + 1);
    }
    b->ws_bytes = std::max(sort_ws_bytes(xo, tiles + 1, (int)b->seg_f_h.size(), PR_F64, true),
                           sort_ws_bytes(xo, max_inst_tiles + 1, max_k, PR_F64, true));
    PB_ALLOC(b->ws, b->ws_bytes);
    // matching tiles
    std::vector<MatchSeg> ms;
    std::vector<int> mt;
    for (int i = 0; i < B; ++i) {
        b->mtile_first.push_back((int)mt.size());
        for (int s = 0; s < sch[i].n_slices; ++s) {
            MatchSeg m{};
            m.base = b->xoff[i] + (int64_t)(s + 1) * n[i];
            m.n = n[i];
            m.qt_row = b->qrow0[i] + s + 1;
            m.qp_row = m.qt_row;
            m.tile0 = (int64_t)mt.size();
            const int nt = (int)((n[i] + MB_TILE - 1) / MB_TILE);
            for (int t = 0; t < nt; ++t) mt.push_back((int)ms.size());
            ms.push_back(m);
        }
        b->mtile_count.push_back((int)mt.size() - b->mtile_first.back());
    }
    b->n_mtiles = (int)mt.size();
    PR_CHECK(upload(b->mseg, ms, st));
    PR_CHECK(upload(b->mtile, mt, st));

    // zeroth iteration, instance by instance
    for (int i = 0; i < B; ++i) {
        const int K = sch[i].n_slices;
        const int64_t ni = n[i], xo_i = b->xoff[i];
        const int r0 = b->qrow0[i];
        PR_CHECK(init_ensemble(&sde[i], seed, b->inst_id[i], ni, b->x[0] + xo_i, b->y[0] + xo_i, st));
        PR_CHECK(restrict_quantiles(b->x[0] + xo_i, PR_F64, ni, 1, b->Q, nullptr, b->q + (int64_t)r0 * (b->Q + 1),
                                    b->rank + xo_i, nullptr, nullptr, nullptr, nullptr, b->ws, st));
        hipLaunchKernelGGL(chain_kernel, dim3(1), dim3(CHAIN_THREADS), lds_chain(b->g), st, (const ChainInst *)b->chain, i,
                           (const CoarseUnit *)b->cu, (const double *)b->E, (const double *)b->q, nullptr, nullptr,
                           b->q, b->g);
        PR_LAUNCHED();
        MatchArgs ma{b->q + (int64_t)(r0 + 1) * (b->Q + 1), b->Q + 1, b->q + (int64_t)r0 * (b->Q + 1), 0,
                     b->rank + xo_i, 0, b->x[0] + xo_i, 0, b->x[0] + xo_i + ni, ni};
        PR_CHECK(match_strided(ma, ni, K, b->Q, PR_F64, st));
        PR_CHECK(restrict_quantiles(b->x[0] + xo_i, PR_F64, ni, K + 1, b->Q, nullptr,
                                    b->qR + (int64_t)r0 * (b->Q + 1), nullptr, nullptr, nullptr, nullptr, nullptr,
                                    b->ws, st));
    }
    // every instance's states [xoff, xoff + (K+1) n) lie inside the buffers
    // and do not overlap the next instance's
    int64_t max_n = 1;
    for (int i = 0; i < B; ++i) {
        const int64_t end = b->xoff[i] + (int64_t)(sch[i].n_slices + 1) * n[i];
        if (b->xoff[i] < 0 || end > xo || (i + 1 < B && end != b->xoff[i + 1])) {
            set_error("state layout of instance %d out of bounds", i);
            return PR_E_INVALID;
        }
        max_n = std::max(max_n, n[i]);
    }
    hipLaunchKernelGGL(spread_time0, dim3((unsigned)std::min<int64_t>((max_n + 255) / 256, 256), (unsigned)B),
                       dim3(256), 0, st, (const InstDev *)b->inst, b->x[0], b->y[0], b->x[1], b->y[1]);
    PR_LAUNCHED();
    PR_HIP(hipStreamSynchronize(st));
    if (flags & PR_AUTOTUNE) {
        PR_CHECK(autotune(b, st));
        PR_CHECK(tune_sort(b, st));
    }
    PR_CHECK(fine_slots(b->tuned, b->persist_blocks));
    build_units(b, b->tuned.block * b->tuned.ppt);
    PR_CHECK(upload(b->units, b->units_h, st));
    for (auto &e : b->ev) PR_HIP(hipEventCreate(&e));
    PR_HIP(hipStreamSynchronize(st));
    return PR_OK;
}

static int capture(Batch *b, int parity, hipStream_t st) {
    const int saved = b->cur;
    b->cur = parity;
    hipGraph_t graph = nullptr;
    PR_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int s = iterate_once(b, 0, st);
    const hipError_t e = hipStreamEndCapture(st, &graph);
    b->cur = saved;
    if (s != PR_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    PR_HIP(e);
    PR_HIP(hipGraphInstantiate(&b->graph[parity], graph, nullptr, nullptr, 0));
    PR_HIP(hipGraphDestroy(graph));
    return PR_OK;
}

}  // namespace pr

using namespace pr;

extern "C" int pr_draw_instances(uint64_t seed, int count, double *out, void *stream) {
    clear_error();
    PR_REQUIRE(count >= 1 && out != nullptr, "count >= 1 and out non-NULL");
    hipLaunchKernelGGL(draw_instances_kernel, dim3((count + 63) / 64), dim3(64), 0, as_stream(stream), out, count,
                       make_key(seed));
    PR_LAUNCHED();
    return PR_OK;
}

extern "C" int pr_parareal_batch_create(int n_inst, const pr_sde *sde, const pr_schedule *sched, const int64_t *n,
                                        const pr_grid *grid, uint64_t seed, const uint32_t *instance, int flags,
                                        void *stream, void **h) {
    clear_error();
    PR_REQUIRE(n_inst >= 1 && n_inst <= 65535, "n_inst must be in [1, 65535]");
    PR_REQUIRE(sde && sched && n && h, "sde, sched, n and h must be non-NULL");
    PR_CHECK(check_grid(grid));
    PR_REQUIRE((flags & ~(PR_REUSE_COARSE | PR_AUTOTUNE)) == 0, "unknown flags");
    for (int i = 0; i < n_inst; ++i) {
        PR_CHECK(check_sde(&sde[i]));
        PR_CHECK(check_schedule(&sched[i]));
        PR_REQUIRE(sde[i].d_fast == 1 && sde[i].precision == PR_F64, "batched instances serve d = 1, FP64");
        PR_REQUIRE(n[i] >= 1 && n[i] <= 0x7FFFFFFFll, "n[%d] must be in [1, 2^31)", i);
        PR_REQUIRE(sched[i].n_slices <= 1023, "at most 1023 slices per instance");
    }
    Batch *b = new Batch();
    const int s = batch_create(n_inst, sde, sched, n, grid, seed, instance, flags, as_stream(stream), b);
    if (s != PR_OK) {
        batch_free(b);
        return s;
    }
    *h = b;
    return PR_OK;
}

extern "C" int pr_parareal_batch_iterate(void *hv, int n_iter, int mode, double *ms_out, void *stream) {
    clear_error();
    PR_REQUIRE(hv != nullptr && n_iter >= 0, "h non-NULL and n_iter >= 0");
    PR_REQUIRE(mode == PR_LAUNCH_BATCHED || mode == PR_LAUNCH_GRAPH || mode == PR_LAUNCH_PER_INSTANCE,
               "unknown launch mode");
    Batch *b = (Batch *)hv;
    hipStream_t st = as_stream(stream);
    PR_REQUIRE(mode != PR_LAUNCH_GRAPH || st != nullptr, "graph capture needs a non-default stream");
    if (mode == PR_LAUNCH_GRAPH)
        for (int p = 0; p < 2; ++p)
            if (!b->graph[p]) PR_CHECK(capture(b, p, st));
    PR_HIP(hipEventRecord(b->ev[0], st));
    for (int it = 0; it < n_iter; ++it) {
        if (mode == PR_LAUNCH_GRAPH) PR_HIP(hipGraphLaunch(b->graph[b->cur], st));
        else PR_CHECK(iterate_once(b, mode == PR_LAUNCH_PER_INSTANCE ? 1 : 0, st));
        if (mode != PR_LAUNCH_PER_INSTANCE) PR_CHECK(sort_new_if_flagged(b, 1 - b->cur, st));
        b->cur = 1 - b->cur;
        b->k += 1;
    }
    PR_HIP(hipEventRecord(b->ev[1], st));
    if (ms_out) {
        PR_HIP(hipEventSynchronize(b->ev[1]));
        float ms = 0.f;
        PR_HIP(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
        *ms_out = ms;
    }
    return PR_OK;
}

extern "C" int pr_parareal_batch_state(void *hv, int inst, int t, void *x, void *y, double *q, void *stream) {
    clear_error();
    PR_REQUIRE(hv != nullptr, "h is NULL");
    Batch *b = (Batch *)hv;
    PR_REQUIRE(inst >= 0 && inst < b->B, "instance out of range");
    PR_REQUIRE(t >= 0 && t <= b->sch[inst].n_slices, "t out of range");
    hipStream_t st = as_stream(stream);
    const int64_t off = b->xoff[inst] + (int64_t)t * b->n[inst];
    if (x) PR_HIP(hipMemcpyAsync(x, b->x[b->cur] + off, sizeof(double) * b->n[inst], hipMemcpyDeviceToDevice, st));
    if (y) PR_HIP(hipMemcpyAsync(y, b->y[b->cur] + off, sizeof(double) * b->n[inst], hipMemcpyDeviceToDevice, st));
    if (q)
        PR_HIP(hipMemcpyAsync(q, b->qR + (int64_t)(b->qrow0[inst] + t) * (b->Q + 1), sizeof(double) * (b->Q + 1),
                              hipMemcpyDeviceToDevice, st));
    return PR_OK;
}

extern "C" int pr_parareal_batch_info(const void *hv, int *tuned_block, int *tuned_ppt, int64_t *units,
                                      int64_t *particle_steps, int *split_sort) {
    clear_error();
    PR_REQUIRE(hv != nullptr, "h is NULL");
    const Batch *b = (const Batch *)hv;
    if (tuned_block) *tuned_block = b->tuned.block;
    if (tuned_ppt) *tuned_ppt = b->tuned.ppt;
    if (split_sort) *split_sort = b->split_sort ? 1 : 0;
    if (units) *units = b->n_units;
    if (particle_steps) {
        int64_t w = 0;
        for (int i = 0; i < b->B; ++i) w += b->n[i] * b->sch[i].total_steps;
        *particle_steps = w;
    }
    return PR_OK;
}

extern "C" int pr_parareal_batch_knot_sorts(const void *hv, int64_t *segments) {
    if (!hv) return -1;
    const Batch *b = (const Batch *)hv;
    if (segments) *segments = b->knot_sort_segs;
    return b->knot_sorts;
}

extern "C" int pr_parareal_batch_destroy(void *h) {
    clear_error();
    batch_free((Batch *)h);
    return PR_OK;
}
