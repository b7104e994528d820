// Device helpers of the coarse propagator shared by the single-instance and
// the batched drivers: the piecewise-linear cdf of a knot vector (Sec. 4.4,
// eq. (discr_cdf) read on the quantile side), its inverse on cell masses
// with the flat-stretch midpoint rule, and pool-adjacent-violators.
#pragma once

#include "pr_internal.hpp"

namespace pr {

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

// Pool-adjacent-violators (equal weights), single thread, in place; L <= cap.
__device__ inline void pava_serial(double *v, int L, double *S, int *Cn) {
#pragma clang fp contract(off)
    int nb = 0;
    for (int i = 0; i < L; ++i) {
        double s = v[i];
        int c = 1;
        while (nb > 0 && S[nb - 1] / (double)Cn[nb - 1] > s / (double)c) {
            s += S[nb - 1];
            c += Cn[nb - 1];
            --nb;
        }
        S[nb] = s;
        Cn[nb] = c;
        ++nb;
    }
    int o = 0;
    for (int b = 0; b < nb; ++b) {
        const double m = S[b] / (double)Cn[b];
        for (int t = 0; t < Cn[b]; ++t) v[o++] = m;
    }
}

}  // namespace pr
