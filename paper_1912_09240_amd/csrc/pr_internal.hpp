// Internal helpers of the HIP library: error reporting, launch checks and the
// device-side counter-based noise (Philox4x32-10 + Box-Muller).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "pr.h"
#include "pr_fastmath.hpp"
#include "pr_normal.hpp"

namespace pr {

// ---------------------------------------------------------------------------
// Errors: every entry point returns a pr_status; the message is thread-local.
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();

#define PR_REQUIRE(cond, ...)                                   \
    do {                                                        \
        if (!(cond)) {                                          \
            ::pr::set_error(__VA_ARGS__);                       \
            return PR_E_INVALID;                                \
        }                                                       \
    } while (0)

#define PR_HIP(call)                                                                 \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) {                                                      \
            ::pr::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),   \
                            __FILE__, __LINE__);                                     \
            return PR_E_HIP;                                                         \
        }                                                                            \
    } while (0)

#define PR_LAUNCHED()                                                                \
    do {                                                                             \
        hipError_t e_ = hipGetLastError();                                           \
        if (e_ != hipSuccess) {                                                      \
            ::pr::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), \
                            __FILE__, __LINE__);                                     \
            return PR_E_HIP;                                                         \
        }                                                                            \
    } while (0)

#define PR_CHECK(expr)               \
    do {                             \
        int s_ = (expr);             \
        if (s_ != PR_OK) return s_;  \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline bool valid_precision(int p) { return p == PR_F64 || p == PR_F32; }
inline bool valid_d(int d) { return d == 1 || d == 2 || d == 3 || d == 4 || d == 8 || d == 16 || d == 32; }

int check_sde(const pr_sde *s);
int check_schedule(const pr_schedule *s);
int check_grid(const pr_grid *g);

// First step of slice n: floor(n S / N), computed without overflow for
// S < 2^63 / N.
__host__ __device__ inline int64_t slice_begin(int64_t S, int N, int n) {
    return (int64_t)((__int128)n * S / N);
}

// A value the caller knows to be equal in every lane, moved to scalar
// registers (the first lane's copy): the slice bounds above come out of a
// 128-bit division done on the vector unit.
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// Noise.  Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
//   (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key advanced by the Weyl increments (k0 + r W0, k1 + r W1 in
// round r).
// ---------------------------------------------------------------------------
struct Block {
    uint32_t w0, w1, w2, w3;
};

// One round.  XOR3 selects a single three-input VALU xor for the words that
// vary across lanes; for the counter layout used here (only the particle
// index varies inside a wave) the first rounds mix mostly wave-uniform words,
// which the compiler keeps on the scalar unit.
template <bool XOR3_0, bool XOR3_2>
__device__ __forceinline__ void philox_round(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3,
                                             uint32_t k0, uint32_t k1) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t h0 = (uint32_t)(p0 >> 32), h1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = XOR3_0 ? __builtin_amdgcn_bitop3_b32(h1, c1, k0, 0x96) : (h1 ^ c1 ^ k0);
    const uint32_t n2 = XOR3_2 ? __builtin_amdgcn_bitop3_b32(h0, c3, k1, 0x96) : (h0 ^ c3 ^ k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
}

__device__ __forceinline__ Block philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    philox_round<false, false>(c0, c1, c2, c3, k0, k1);
    philox_round<false, false>(c0, c1, c2, c3, k0 + W0, k1 + W1);
    philox_round<false, false>(c0, c1, c2, c3, k0 + 2 * W0, k1 + 2 * W1);
    philox_round<true, false>(c0, c1, c2, c3, k0 + 3 * W0, k1 + 3 * W1);
#pragma unroll
    for (uint32_t r = 4; r < 10; ++r) philox_round<true, true>(c0, c1, c2, c3, k0 + r * W0, k1 + r * W1);
    return Block{c0, c1, c2, c3};
}

struct Key {
    uint32_t k0, k1;
};
inline Key make_key(uint64_t seed) { return Key{(uint32_t)seed, (uint32_t)(seed >> 32)}; }

__device__ __forceinline__ Block noise_block(Key key, uint32_t inst, uint32_t tag, uint32_t m,
                                             uint32_t p, uint32_t j) {
    return philox(m, p, (tag << 16) | j, inst, key.k0, key.k1);
}

// 53-bit uniforms: u1 in (0, 1] (never 0, so log is finite), u2 in [0, 1).
__device__ __forceinline__ void uniforms53(const Block &b, double &u1, double &u2) {
#pragma clang fp contract(off)
    const double a = (double)(b.w0 >> 5) * 67108864.0 + (double)(b.w1 >> 6);
    const double c = (double)(b.w2 >> 5) * 67108864.0 + (double)(b.w3 >> 6);
    u1 = (a + 0.5) * 0x1p-53;
    u2 = c * 0x1p-53;
}

// Box-Muller pair of one block, FP64 (bit layout and elementary functions in
// pr_normal.hpp; the tables must be in LDS, see load_noise_tab).
__device__ __forceinline__ void box_muller(const Block &b, const NoiseTab &tab, double &z0, double &z1) {
    normal_pair_of_words(b.w0, b.w1, b.w2, b.w3, tab, z0, z1);
}

// FP32 variant with the same bits at single precision: u from the top 24
// bits of w0, the angle from bits 4..31 of w2 (no tables).
__device__ __forceinline__ void box_muller_f32(const Block &b, float &z0, float &z1) {
    const float u1 = ((float)(b.w0 >> 8) + 0.5f) * 0x1p-24f;
    const float t = ((float)((b.w2 >> 4) & 255u) + (float)(b.w2 >> 12) * 0x1p-20f) * 0x1p-7f;
    const float r = sqrtf(-2.0f * logf(u1));
    float s, c;
    sincospif(t, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// Orderable 64-bit key of a double: unsigned order == numeric order,
// -0.0 before +0.0.
__device__ __forceinline__ uint64_t key_of(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint64_t mask = (uint64_t)((int64_t)b >> 63) | 0x8000000000000000ull;
    return b ^ mask;
}
__device__ __forceinline__ double value_of(uint64_t k) {
    const uint64_t b = (k & 0x8000000000000000ull) ? (k ^ 0x8000000000000000ull) : ~k;
    return __longlong_as_double((long long)b);
}
__device__ __forceinline__ uint32_t key_of(float x) {
    const uint32_t b = (uint32_t)__float_as_uint(x);
    const uint32_t mask = (uint32_t)((int32_t)b >> 31) | 0x80000000u;
    return b ^ mask;
}
__device__ __forceinline__ double value_of(uint32_t k) {
    const uint32_t b = (k & 0x80000000u) ? (k ^ 0x80000000u) : ~k;
    return (double)__uint_as_float(b);
}

// Matching that preserves the fast marginal (Sec. 5.1, eq. (transformation))
// of one particle: its prior value x at the mid-rank cdf value
// u = (rank + 1/2)/P moved by the linear interpolant, at u, of the knot
// differences dk = q_target - q_prior on the levels j/Q.  Every kernel that
// needs a matched value calls this, so they agree bit for bit.
template <typename T>
__device__ __forceinline__ T matched_value(T x, uint64_t rank, const double *dk, double nd, double Q) {
#pragma clang fp contract(off)
    const double u = ((double)rank + 0.5) / nd;
    const double uq = u * Q;
    double jf = floor(uq);
    jf = jf < Q - 1.0 ? jf : Q - 1.0;
    const int j = (int)jf;
    const double w = uq - jf;
    const double delta = (1.0 - w) * dk[j] + w * dk[j + 1];
    return (T)((double)x + delta);
}

// ---------------------------------------------------------------------------
// Internal entry points shared between translation units (no validation).
// ---------------------------------------------------------------------------
// Per-segment strides (in elements) let one prior serve several targets
// (stride 0), as in the zeroth iteration where every slice is matched
// against the initial ensemble.
struct MatchArgs {
    const double *qt;
    int64_t qt_stride;
    const double *qp;
    int64_t qp_stride;
    const uint32_t *rank;
    int64_t rank_stride;
    const void *xin;
    int64_t xin_stride;
    void *xout;
    int64_t xout_stride;
};
int match_strided(const MatchArgs &a, int64_t n, int k, int nq, int precision, hipStream_t st);

// Knots of the k matched ensembles X = M(Xbar) (n particles each, matched
// with the knot rows qt, qp as by match_strided) straight from the sorted
// keys that the last restrict_quantiles call on Xbar left in ws, without a
// sort of X: *flag (device) is set where some order statistic could not be
// isolated, and the knots are then to be taken by restrict_quantiles.
// Returns PR_E_UNSUPPORTED (nothing launched) where ws has no room for the
// chunk extremes.
int matched_knots(const void *ws, int precision, int64_t n, int k, int nq, const double *qt, int64_t qt_stride,
                  const double *qp, int64_t qp_stride, double *q, int *flag, hipStream_t st);

// The same for ensembles of unequal lengths (FP64) whose sort used a segment
// table: segment s of the table holds ensemble s (its keys at base, n of
// them), matched with knot rows qt_row, qp_row, its knots going to q_row;
// ch0, gr0 number its first chunk (64 ranks) and group (4096 ranks) among
// all segments' (host-computed prefix sums).  group_seg maps every group to
// its segment.  Scratch: the key buffer of ws that the sort did not end in.
struct MkSeg {
    int64_t base, n, ch0, gr0;
    int qt_row, qp_row, q_row, pad;
};
int matched_knots_segments(const void *ws, int64_t total_keys, int nseg, const MkSeg *segs, const int *group_seg,
                           int64_t total_chunks, int64_t total_groups, int nq, const double *qt, const double *qp,
                           double *q, int *flag, int *segflag, hipStream_t st);

// x_in/y_in and x_out/y_out may alias (in place).
int fine_propagate(const pr_sde *sde, const pr_schedule *sch, uint64_t seed, uint32_t inst, int64_t n,
                   int slice_first, int slice_count, const void *x_in, const void *y_in, void *x_out,
                   void *y_out, hipStream_t st);
int init_ensemble(const pr_sde *sde, uint64_t seed, uint32_t inst, int64_t n, void *x, void *y, hipStream_t st);

// Segments of one sort call.  Equal lengths: segs == NULL, segment s starts
// at s * n.  Unequal lengths: a segment table and the segment of every tile
// (tiles ordered by segment).
struct SortSeg {
    int64_t base;   // element offset of the segment in the value/rank arrays
    int64_t n;      // length
    int64_t tile0;  // index of its first tile
    int32_t nblk;   // number of tiles
    int32_t qrow;   // knot row of the segment
};
struct SortLayout {
    int64_t n;             // equal lengths: keys per segment
    int nblk;              // equal lengths: tiles per segment
    int nseg;
    const SortSeg *segs;   // unequal lengths: device table [nseg]
    const int *tile_seg;   // unequal lengths: device table [tiles]
    const int *guard;      // device flag or NULL: while it reads 0 every kernel of the sort returns at once
    int64_t max_n;         // unequal lengths: the longest segment (0 if not known)
    int64_t min_n;         // unequal lengths: the shortest segment (0 if not known)
};
int64_t sort_tiles(int64_t n);
// Whether an FP64 ensemble of n keys is sorted by splitters and buckets
// (with ranks or the permutation asked for) rather than by radix passes.
bool splitter_sorts(int64_t n);
size_t sort_ws_bytes(int64_t total_keys, int64_t total_tiles, int nseg, int precision, bool payload);
int restrict_segments(const void *x, int precision, const SortLayout &L, int64_t total_keys, int64_t total_tiles,
                      int nq, double *q, uint32_t *rank, void *ws, hipStream_t st);
// restrict_quantiles of k equal segments for knots only, every kernel
// returning at once while *guard reads 0 (a sort that runs only where the
// device decides it is needed, launched unconditionally).
int restrict_knots_guarded(const void *x, int precision, int64_t n, int k, int nq, double *q, void *ws,
                           const int *guard, hipStream_t st);
size_t restrict_ws(int64_t n, int k, int precision);
int restrict_quantiles(const void *x, int precision, int64_t n, int k, int nq, const pr_grid *hg, double *q,
                       uint32_t *rank, uint32_t *perm, double *xs, double *mom, uint32_t *hist, void *ws,
                       hipStream_t st);

struct Coarse;
int coarse_create(const pr_sde *sde, const pr_schedule *sch, const pr_grid *grid, hipStream_t st, Coarse **out);
int coarse_step(const Coarse *c, int first, int count, const double *q_in, int in_stride, double *q_out,
                int out_stride, double *rho_out, hipStream_t st);
int coarse_jump(const Coarse *c, int n, const double *q_cur, const double *qf, const double *qcs, double *q_next,
                double *qc_out, hipStream_t st);
int coarse_apply(const Coarse *c, int first, int count, const double *rho_in, double *rho_out, hipStream_t st);
void coarse_free(Coarse *c);

}  // namespace pr
