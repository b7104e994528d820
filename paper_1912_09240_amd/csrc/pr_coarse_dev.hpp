// Device helpers of the coarse propagator shared by the single-instance and
// the batched drivers: the piecewise-linear cdf of a knot vector (Sec. 4.4,
// eq. (discr_cdf) read on the quantile side), its inverse on cell masses
// with the flat-stretch midpoint rule, and pool-adjacent-violators.
#pragma once

#include "pr_internal.hpp"

namespace pr {

// One lane's share of a row-vector product (elements lane, lane + 64, ...):
// the loads of the row run eight ahead of the multiply-adds, whose order stays
// the element order, so the sum is that of the plain loop.
__device__ __forceinline__ double lane_row_dot(const double *__restrict__ row, const double *v, int n, int lane) {
    double acc = 0.0;
    int j = lane;
    for (; j + 7 * 64 < n; j += 8 * 64) {
        double e[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) e[u] = row[j + u * 64];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma(e[u], v[j + u * 64], acc);
    }
    for (; j < n; j += 64) acc = fma(row[j], v[j], acc);
    return acc;
}

// The lane's shares of R rows at once (row k at rows[k]): every row's
// multiply-adds run in the element order of lane_row_dot, so each sum has
// its bits; the loads of U elements of all R rows are issued before any of
// them is used, R U loads in flight per lane.
template <int R, int U>
__device__ __forceinline__ void lane_rows_dot(const double *const *rows, const double *v, int n, int lane,
                                              double *acc) {
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = 0.0;
    for (int j0 = lane; j0 < n; j0 += 64 * U) {
        double e[R][U];
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = j0 + u * 64;
                e[k][u] = j < n ? rows[k][j] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + u * 64;
            if (j < n) {
                const double vj = v[j];
#pragma unroll
                for (int k = 0; k < R; ++k) acc[k] = fma(e[k][u], vj, acc[k]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Knots -> cell masses (H).  c(x) = 0 for x <= q_0, 1 for x > q_Q, else
// (j + (x - q_j)/(q_{j+1} - q_j))/Q with j the largest index with q_j < x
// (a repeated knot is a jump; c(x) = P(X < x)).  rho_i = c(x_{i+1}) - c(x_i),
// the mass beyond the grid going to the end cells.
// ---------------------------------------------------------------------------
struct GridDev {
    int cells, nq;
    double lo, h;
};

__device__ __forceinline__ double edge_at(const GridDev &g, int i) {
#pragma clang fp contract(off)
    return g.lo + (double)i * g.h;
}

__device__ inline double cdf_knots(const double *q, int nq, double x) {
#pragma clang fp contract(off)
    if (x <= q[0]) return 0.0;
    if (x > q[nq]) return 1.0;
    int lo = 0, hi = nq;  // q[lo] < x <= q[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (q[mid] < x) lo = mid;
        else hi = mid;
    }
    const double t = (x - q[lo]) / (q[lo + 1] - q[lo]);
    return ((double)lo + t) / (double)nq;
}

// Cell masses -> knots (Qf) of the piecewise-linear cdf with cumulative
// masses C_i (left to right); level p_j C_I.  A level hit on a flat stretch
// gives its midpoint; the end knots are the grid ends.  Runs inside one
// block; C must hold cells + 1 doubles of LDS.
__device__ inline void masses_to_knots_block(const double *rho, double *C, const GridDev &g, double *q) {
#pragma clang fp contract(off)
    // C_{i+1} = C_i + rho_i strictly left to right (the same additions as a
    // serial loop), done by one wave: each lane holds 16 consecutive masses
    // in registers and the running sum is handed from lane to lane.
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        if (lane == 0) C[0] = 0.0;
        double carry = 0.0;
        for (int base = 0; base < g.cells; base += 1024) {
            double v[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int idx = base + lane * 16 + i;
                v[i] = idx < g.cells ? rho[idx] : 0.0;
            }
            double mine = 0.0;
            for (int l = 0; l < 64; ++l) {
                if (lane == l) {
                    double acc = carry;
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        if (base + lane * 16 + i < g.cells) acc = acc + v[i];
                        v[i] = acc;
                    }
                    mine = acc;
                }
                carry = __shfl(mine, l);
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int idx = base + lane * 16 + i;
                if (idx < g.cells) C[idx + 1] = v[i];
            }
        }
    }
    __syncthreads();
    const double tot = C[g.cells];
    for (int j = threadIdx.x; j <= g.nq; j += blockDim.x) {
        double v;
        if (j == 0) {
            v = edge_at(g, 0);
        } else if (j == g.nq) {
            v = edge_at(g, g.cells);
        } else {
            const double ct = ((double)j / (double)g.nq) * tot;
            int lo = -1, hi = g.cells;  // first i with C_i >= ct: C[lo] < ct <= C[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (C[mid] >= ct) hi = mid;
                else lo = mid;
            }
            const int i1 = hi;
            if (C[i1] > ct) {
                const int i = i1 - 1;
                const double e0 = edge_at(g, i), e1 = edge_at(g, i + 1);
                double x = e0 + (ct - C[i]) / rho[i] * g.h;
                x = x > e0 ? x : e0;
                v = x < e1 ? x : e1;
            } else {
                int lo2 = i1, hi2 = g.cells + 1;  // last i with C_i <= ct: C[lo2] <= ct < C[hi2]
                while (hi2 - lo2 > 1) {
                    const int mid = (lo2 + hi2) >> 1;
                    if (C[mid] <= ct) lo2 = mid;
                    else hi2 = mid;
                }
                v = 0.5 * (edge_at(g, i1) + edge_at(g, lo2));
            }
        }
        q[j] = v;
    }
}

// The value of v in lane l (uniform l) of the wave.
__device__ __forceinline__ double lane_value(double v, int l) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Whether the rounded mean a/ca exceeds the rounded mean b/cb (counts >= 1).
// Where the cross products a*cb and b*ca differ by more than 2^-49 of their
// magnitudes (plus 2^-1000), the exact means differ by more than 2^-50 of
// theirs, more than the two roundings of the divisions can close, so the
// rounded means compare as the exact ones do; otherwise (and for inf or NaN)
// both divisions are taken and compared.  The result is that of comparing
// the two rounded quotients in every case.
__host__ __device__ inline bool mean_above(double a, int ca, double b, int cb) {
#pragma clang fp contract(off)
    const double x = a * (double)cb, y = b * (double)ca;
    const double d = x - y, tol = (fabs(x) + fabs(y)) * 0x1p-49 + 0x1p-1000;
    if (d > tol) return true;
    if (-d > tol) return false;
    return a / (double)ca > b / (double)cb;
}

// Pool-adjacent-violators (equal weights) over the stretch [lo, hi) of v
// alone, as if it started the input, with the same additions and the same
// outcome of every comparison as the textbook stack form: a new value starts
// a pool (sum s, count c); while the pool below has a larger rounded mean
// S/C it is merged (s = s + S, c = c + C).  vio: the violations v[j] >
// v[j+1] inside the stretch, increasing (positions absolute, at least one).
//
// The pool on top (T) and the pool just below it (B) are held in registers;
// of the pools under T only those of more than one value are stored, in
// position order, at S[lo + k] and SC[lo + k] = start << 16 | count (B, when
// it has more than one value, is the last of them); a pool of one value is
// read back from v.  A run of values that each merge into T (a decreasing
// run) thus touches only v.  When T is a single value, nothing merges until
// the next violation: the values in between stay single pools and are
// skipped.  Returns the number of stored pools.  *fm receives the smallest
// of the means that the pool holding lo takes (v[lo] first, then after
// every merge that reaches lo): the values the serial pass over a longer
// input would compare with the mean of the last pool before the stretch.
// *lm receives the mean of the pool holding hi - 1.
//
// WAVE: called by a whole wave with the same arguments (every lane runs the
// same scalar steps on the same values).  Where T holds more than one value
// and the next value merges into it while B stays below, the wave takes the
// run ahead at once: lane j adds v[i + j] to T's sum after the lanes before
// it, in the serial order, and checks the two comparisons the serial pass
// would make for that value; the longest prefix of lanes that pass is
// committed (windows of 8 values, doubling up to 64 while whole windows
// pass).  A decreasing run of L values then costs about L / 64 windows
// instead of L serial steps.
template <bool WAVE = false>
__host__ __device__ inline int pava_sparse_range(const double *v, int lo, int hi, const int *vio, int nv,
                                                 double *S, int *SC, double *fm, double *lm) {
#pragma clang fp contract(off)
    int nb = 0, vi = 0;
    int win = 8;
    double fmin_ = v[lo];
    int i = vio[0];
    double tS = v[i], bS = 0.0;
    int tC = 1, tSt = i, bC = 1, bSt = i - 1;
    if (i > lo) bS = v[i - 1];
    ++i;
    double vcur = v[i < hi ? i : hi - 1];
    while (i < hi) {
        if (tC == 1) {
            // first violation at or after i - 1 (a decreasing run leaves a
            // long stretch of consumed ones behind)
            if constexpr (WAVE) {
                // 64 entries per look, one per lane
                const int lane = (int)(threadIdx.x & 63);
                while (true) {
                    const int idx = vi + lane;
                    const uint64_t bm = __ballot(idx >= nv || vio[idx] >= i - 1);
                    if (bm) {
                        vi += __builtin_ctzll(bm);
                        break;
                    }
                    vi += 64;
                }
                if (vi > nv) vi = nv;
            } else {
                int lo2 = vi, hi2 = nv;  // binary search
                while (lo2 < hi2) {
                    const int mid = (lo2 + hi2) >> 1;
                    if (vio[mid] < i - 1) lo2 = mid + 1;
                    else hi2 = mid;
                }
                vi = lo2;
            }
            if (vi == nv) break;  // non-decreasing from v[i-1] on
            const int jn = vio[vi];
            if (jn > i - 1) {
                tSt = jn;
                tS = v[jn];
                bSt = jn - 1;  // a single value: the values since i - 1 stay single
                bS = v[jn - 1];
                bC = 1;
                i = jn + 1;
                vcur = v[i];
            }
        }
        if constexpr (WAVE) {
            if (tC > 1 && mean_above(tS, tC, vcur, 1) && (tSt == lo || !mean_above(bS, bC, vcur + tS, tC + 1))) {
                const int lane = (int)(threadIdx.x & 63);
                const int m = hi - i < win ? hi - i : win;
                const double ve = lane < m ? v[i + lane] : 0.0;  // one load for the window
                double acc = tS, prev = tS;  // T's sum before and after this lane's value
                for (int k = 0; k < m; ++k) {
                    const double vk = lane_value(ve, k);
                    if (k <= lane) {
                        prev = acc;
                        acc = vk + acc;
                    }
                }
                const int cb = tC + lane;
                const bool ok = lane < m && mean_above(prev, cb, ve, 1) &&
                                (tSt == lo || !mean_above(bS, bC, acc, cb + 1));
                const uint64_t bad = __ballot(!ok);
                const int f = bad ? __builtin_ctzll(bad) : 64;  // >= 1: lane 0 passes
                if (tSt == lo) {
                    double mm = lane < f ? acc / (double)(cb + 1) : INFINITY;
                    for (int off = 32; off >= 1; off >>= 1) {
                        const double o = __shfl_xor(mm, off);
                        mm = o < mm ? o : mm;
                    }
                    if (mm < fmin_) fmin_ = mm;
                }
                tS = lane_value(acc, f - 1);
                tC += f;
                i += f;
                win = f == m ? (win < 64 ? 2 * win : 64) : 8;
                vcur = v[i < hi ? i : hi - 1];
                continue;
            }
            win = 8;
        }
        double s = vcur;
        vcur = v[i + 1 < hi ? i + 1 : i];  // the next value, loaded ahead
        int c = 1, st = i;
        if (mean_above(tS, tC, s, c)) {
            s = s + tS;
            c = c + tC;
            st = tSt;
            if (st == lo) {
                const double m = s / (double)c;
                if (m < fmin_) fmin_ = m;
            }
            while (st != lo && mean_above(bS, bC, s, c)) {
                s = s + bS;
                c = c + bC;
                st = bSt;
                if (bC > 1) --nb;  // B was the last stored pool
                if (st == lo) {
                    const double m = s / (double)c;
                    if (m < fmin_) fmin_ = m;
                } else {
                    const int k = lo + (nb > 0 ? nb - 1 : 0);
                    const int sc = SC[k];
                    const double sv = S[k], vv = v[st - 1];
                    if (nb > 0 && (sc >> 16) + (sc & 0xFFFF) == st) {
                        bS = sv;
                        bC = sc & 0xFFFF;
                        bSt = sc >> 16;
                    } else {
                        bS = vv;
                        bC = 1;
                        bSt = st - 1;
                    }
                }
            }
            tS = s;
            tC = c;
            tSt = st;
        } else {
            if (tC > 1) {
                S[lo + nb] = tS;
                SC[lo + nb] = (tSt << 16) | tC;
                ++nb;
            }
            bS = tS;
            bC = tC;
            bSt = tSt;
            tS = s;
            tC = 1;
            tSt = i;
        }
        ++i;
    }
    *lm = (i - 1 == hi - 1) ? tS / (double)tC : v[hi - 1];
    if (tC > 1) {
        S[lo + nb] = tS;
        SC[lo + nb] = (tSt << 16) | tC;
        ++nb;
    }
    *fm = fmin_;
    return nb;
}

// The same pass over the whole input v[0..L).
__host__ __device__ inline void pava_sparse(const double *v, int L, const int *vio, int nv, double *S, int *SC,
                                            int *npools) {
    double fm, lm;
    *npools = pava_sparse_range(v, 0, L, vio, nv, S, SC, &fm, &lm);
}

// Pool-adjacent-violators over v[0..L) by the whole block from its known
// violations vio[0..nv) (increasing), with the arithmetic of the serial
// stack form.  The input is cut where every value before is below every
// value after (no pool can reach across such a cut); the stretches between
// cuts that hold violations run pava_sparse_range, one wave each.  Where
// the last pool of a stretch has a mean above a value the first pool of the
// next one takes (rounding can put a pool's mean above its largest value),
// the serial pass would have merged across the cut: those cuts are dropped
// and the stretches run again, until no cut is crossed -- then the pools are
// those of the serial pass, sums and means bit for bit.  At most PAVA_MAXC
// stretches (neighbours beyond that are joined).  LDS: S [L] doubles, SC [L]
// ints (first the last cut at or before every position), and the stretch
// tables.
constexpr int PAVA_MAXC = 512;

struct PavaChunks {
    int cb[PAVA_MAXC + 1];  // stretch bounds
    int fv[PAVA_MAXC + 1];  // first violation of each stretch
    int np[PAVA_MAXC];      // stored pools of each stretch
    int pst[PAVA_MAXC + 1];  // number of the first of them over all stretches
    double fm[PAVA_MAXC], lm[PAVA_MAXC];
    double wmax[16], wmin[16];
    int nc, drop, wsum[16];
};

__device__ inline void pava_block_chunked(double *v, int L, const int *vio, int nv, double *S, int *SC,
                                          PavaChunks &pc) {
    const int nt = (int)blockDim.x, tid = (int)threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    // Cuts: positions b with max(v[0..b)) < min(v[b..L)), where no pool can
    // reach across.  Every thread takes a contiguous run of the values.
    const int per = (L + nt - 1) / nt;
    const int j0 = min(tid * per, L), j1 = min(j0 + per, L);
    {
        double cmax = -INFINITY, cmin = INFINITY;
        for (int j = j0; j < j1; ++j) {
            cmax = fmax(cmax, v[j]);
            cmin = fmin(cmin, v[j]);
        }
        // exclusive prefix max and exclusive suffix min over the threads' runs
        double pmx = cmax, smn = cmin;
        for (int off = 1; off < 64; off <<= 1) {
            const double u = __shfl_up(pmx, off), d = __shfl_down(smn, off);
            if (lane >= off) pmx = fmax(pmx, u);
            if (lane + off < 64) smn = fmin(smn, d);
        }
        if (lane == 63) pc.wmax[w] = pmx;
        if (lane == 0) pc.wmin[w] = smn;
        __syncthreads();
        double before = __shfl_up(pmx, 1), after = __shfl_down(smn, 1);
        if (lane == 0) before = -INFINITY;
        if (lane == 63) after = INFINITY;
        for (int k = 0; k < nt / 64; ++k) {
            if (k < w) before = fmax(before, pc.wmax[k]);
            if (k > w) after = fmin(after, pc.wmin[k]);
        }
        // cut flags of the run: SC[b] = b at a cut, else 0
        double run_max = before;
        for (int b = j0; b < j1; ++b) {
            double suf = after;
            for (int j = j1 - 1; j >= b; --j) suf = fmin(suf, v[j]);
            SC[b] = (b > 0 && run_max < suf) ? b : 0;
            run_max = fmax(run_max, v[b]);
        }
        __syncthreads();
        // SC[j] = the last cut at or before j: inclusive prefix max
        int rmx = 0;
        for (int j = j0; j < j1; ++j) rmx = max(rmx, SC[j]);
        int inc = rmx;
        for (int off = 1; off < 64; off <<= 1) {
            const int u = __shfl_up(inc, off);
            if (lane >= off) inc = max(inc, u);
        }
        if (lane == 63) pc.wsum[w] = inc;
        __syncthreads();
        int carry = __shfl_up(inc, 1);
        if (lane == 0) carry = 0;
        for (int k = 0; k < w; ++k) carry = max(carry, pc.wsum[k]);
        for (int j = j0; j < j1; ++j) {
            carry = max(carry, SC[j]);
            SC[j] = carry;
        }
        __syncthreads();
    }
    // stretches: a new one at every violation whose last cut differs from its
    // predecessor's; at most PAVA_MAXC of them, evenly
    {
        const int fper = (nv + nt - 1) / nt;
        const int f0 = tid * fper, f1 = min(f0 + fper, nv);
        int cnt = 0;
        for (int f = f0; f < f1; ++f) cnt += (f == 0 || SC[vio[f]] != SC[vio[f - 1]]) ? 1 : 0;
        int inc = cnt;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(inc, off);
            if (lane >= off) inc += t;
        }
        if (lane == 63) pc.wsum[w] = inc;
        __syncthreads();
        int base = inc - cnt, total = 0;
        for (int k = 0; k < nt / 64; ++k) {
            if (k < w) base += pc.wsum[k];
            total += pc.wsum[k];
        }
        const int stride = (total + PAVA_MAXC - 1) / PAVA_MAXC;
        for (int f = f0; f < f1; ++f)
            if (f == 0 || SC[vio[f]] != SC[vio[f - 1]]) {
                if (base % stride == 0) {
                    const int k = base / stride;
                    pc.fv[k] = f;
                    pc.cb[k] = f == 0 ? 0 : SC[vio[f]];
                }
                ++base;
            }
        __syncthreads();
        if (tid == 0) {
            const int nc = (total + stride - 1) / stride;
            pc.nc = nc;
            pc.cb[nc] = L;
            pc.fv[nc] = nv;
        }
        __syncthreads();
    }
    while (true) {
        const int nc = pc.nc;
        for (int k = w; k < nc; k += nt / 64) {  // one wave per stretch
            double fm, lm;
            const int np = pava_sparse_range<true>(v, pc.cb[k], pc.cb[k + 1], vio + pc.fv[k],
                                                   pc.fv[k + 1] - pc.fv[k], S, SC, &fm, &lm);
            if (lane == 0) {
                pc.np[k] = np;
                pc.fm[k] = fm;
                pc.lm[k] = lm;
            }
        }
        __syncthreads();
        // keep cut k (1 <= k < nc) unless the serial pass would cross it
        const int per = (nc + nt - 1) / nt;
        const int k0 = tid * per, k1 = min(k0 + per, nc);
        int cnt = 0;
        for (int k = k0; k < k1; ++k) cnt += (k == 0 || !(pc.lm[k - 1] > pc.fm[k])) ? 1 : 0;
        int inc = cnt;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(inc, off);
            if (lane >= off) inc += t;
        }
        if (lane == 63) pc.wsum[w] = inc;
        __syncthreads();
        int base = inc - cnt, total = 0;
        for (int k = 0; k < nt / 64; ++k) {
            if (k < w) base += pc.wsum[k];
            total += pc.wsum[k];
        }
        if (total == nc) break;  // every cut holds (uniform: total is the block's sum)
        // compact the kept cuts in place: kept cut k moves to base <= k, so
        // read every kept value before any write
        int keep_cb[8], keep_fv[8], nk = 0;
        for (int k = k0; k < k1 && nk < 8; ++k)
            if (k == 0 || !(pc.lm[k - 1] > pc.fm[k])) {
                keep_cb[nk] = pc.cb[k];
                keep_fv[nk] = pc.fv[k];
                ++nk;
            }
        __syncthreads();
        for (int t = 0; t < nk; ++t) {
            pc.cb[base + t] = keep_cb[t];
            pc.fv[base + t] = keep_fv[t];
        }
        if (tid == 0) {
            pc.nc = total;
            pc.cb[total] = L;
            pc.fv[total] = nv;
        }
        __syncthreads();
    }
    // write the means of the stored pools of every stretch, one wave per
    // pool: the pools numbered through an exclusive scan of their counts
    const int nc = pc.nc;
    {
        const int per = (nc + nt - 1) / nt;
        const int k0 = min(tid * per, nc), k1 = min(k0 + per, nc);
        int cnt = 0;
        for (int k = k0; k < k1; ++k) cnt += pc.np[k];
        int inc = cnt;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(inc, off);
            if (lane >= off) inc += t;
        }
        if (lane == 63) pc.wsum[w] = inc;
        __syncthreads();
        int base = inc - cnt, total = 0;
        for (int k = 0; k < nt / 64; ++k) {
            if (k < w) base += pc.wsum[k];
            total += pc.wsum[k];
        }
        for (int k = k0; k < k1; ++k) {
            pc.pst[k] = base;
            base += pc.np[k];
        }
        if (tid == 0) pc.pst[nc] = total;
        __syncthreads();
    }
    const int total = pc.pst[nc], wl = min(64, nt - 64 * w);  // lanes of this wave
    for (int g = w; g < total; g += (nt + 63) / 64) {
        int a = 0, b = nc;  // the stretch holding pool g: pst[a] <= g < pst[b]
        while (b - a > 1) {
            const int mid = (a + b) >> 1;
            if (pc.pst[mid] <= g) a = mid;
            else b = mid;
        }
        const int idx = pc.cb[a] + (g - pc.pst[a]);
        const int cq = SC[idx] & 0xFFFF, st = SC[idx] >> 16;
        const double mean = S[idx] / (double)cq;
        for (int t = lane; t < cq; t += wl) v[st + t] = mean;
    }
    __syncthreads();
}

// Pool-adjacent-violators over v[0..L) (L < 65536) by the whole block, with
// the arithmetic of the serial stack form: the violations v[j] > v[j+1] are found
// in parallel; without any, v is already the result; otherwise one thread
// builds the pools with pava_sparse and the block writes their means.  LDS:
// S [L] doubles, SC and vio [L] ints.  Every thread of the block calls it.
__device__ inline void pava_block(double *v, int L, double *S, int *SC, int *vio) {
#pragma clang fp contract(off)
    __shared__ int wsum[16], nbad, npools;
    const int nt = (int)blockDim.x;
    const int per = (L + nt - 1) / nt;
    const int j0 = (int)threadIdx.x * per, j1 = min(j0 + per, L - 1);
    int cnt = 0;
    for (int j = j0; j < j1; ++j) cnt += v[j] > v[j + 1] ? 1 : 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = cnt;
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(inc, off);
        if (lane >= off) inc += t;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int base = inc - cnt;
    for (int k = 0; k < w; ++k) base += wsum[k];
    for (int j = j0; j < j1; ++j)
        if (v[j] > v[j + 1]) vio[base++] = j;
    if ((int)threadIdx.x == nt - 1) nbad = base;
    __syncthreads();
    if (nbad == 0) return;
    if (w == 0) {  // the whole first wave runs the pass
        double fm, lm;
        const int np = pava_sparse_range<true>(v, 0, L, vio, nbad, S, SC, &fm, &lm);
        if (lane == 0) npools = np;
    }
    __syncthreads();
    const int wl = min(64, nt - 64 * w);  // lanes of this wave
    for (int q = w; q < npools; q += (nt + 63) / 64) {  // one wave per pool
        const int cq = SC[q] & 0xFFFF, st = SC[q] >> 16;
        const double mean = S[q] / (double)cq;
        for (int t = lane; t < cq; t += wl) v[st + t] = mean;
    }
    __syncthreads();
}

}  // namespace pr
