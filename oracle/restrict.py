"""Oracle, restriction: empirical quantiles, ranks, moments, histogram.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

Follows Sec. 3.2.2 (restriction R = R2 o R1: drop the fast variable, then
measure the empirical law of the slow one), Sec. 4.4 (quantile function
q = c^-1, support-end and flat-part rules, empirical cdf with strict <) and
Sec. 2.1.3 eq. (MCestimator) for moments with equal weights W = 1/P.
"""
import math

import numpy as np


def orderable_key(x):
    """FP64 -> uint64 whose unsigned order is the numeric order of x
    (negative: all bits flipped; non-negative: sign bit set).  -0.0 orders
    before +0.0."""
    b = np.ascontiguousarray(x, dtype=np.float64).view(np.uint64)
    neg = (b >> np.uint64(63)) == np.uint64(1)
    return np.where(neg, ~b, b | np.uint64(0x8000000000000000))


def sort_ranks(x):
    """Stable ascending order by (key, particle index).

    Returns perm (perm[i] = particle at sorted position i), rank
    (rank[perm[i]] = i) and the sorted values xs."""
    key = orderable_key(x)
    perm = np.argsort(key, kind="stable").astype(np.uint32)
    rank = np.empty(len(x), dtype=np.uint32)
    rank[perm] = np.arange(len(x), dtype=np.uint32)
    xs = np.asarray(x, dtype=np.float64)[perm]
    return perm, rank, xs


def hazen_knots(xs, n_q):
    """Quantile knots at p_j = j/Q, j = 0..Q, of the sorted sample xs with
    the midpoint (Hazen) convention: position t = p_j N - 1/2 between order
    statistics.  At t <= 0 the knot is the minimum and at t >= N-1 the maximum
    (support-end rule of Sec. 4.4 applied to the empirical law); when p_j N is
    an integer the knot is the average of the two straddling order
    statistics, i.e. the flat-part midpoint rule of Sec. 4.4.  An interpolated
    value never leaves [xs[r], xs[r+1]]."""
    xs = np.asarray(xs, dtype=np.float64)
    N = xs.shape[0]
    q = np.empty(n_q + 1, dtype=np.float64)
    for j in range(n_q + 1):
        t = (j * N) / n_q - 0.5
        if t <= 0.0:
            q[j] = xs[0]
        elif t >= N - 1:
            q[j] = xs[N - 1]
        else:
            r = int(math.floor(t))
            f = t - r
            v = xs[r] + f * (xs[r + 1] - xs[r])
            q[j] = min(v, xs[r + 1])
    return q


def hazen_at(xs, p):
    """The same convention at one level p in [0, 1] (observables of the
    differentiated form).  Returns (value, r, f) with the interpolation
    position; r = -1 flags a clamped end."""
    xs = np.asarray(xs, dtype=np.float64)
    N = xs.shape[0]
    t = p * N - 0.5
    if t <= 0.0:
        return xs[0], 0, 0.0
    if t >= N - 1:
        return xs[N - 1], N - 1, 0.0
    r = int(math.floor(t))
    f = t - r
    return min(xs[r] + f * (xs[r + 1] - xs[r]), xs[r + 1]), r, f


def moments(x):
    """Monte Carlo estimates (1/P) sum_p x_p^m, m = 1..4 (eq. (MCestimator) with
    W = 1/P), each sum correctly rounded (math.fsum)."""
    x = np.asarray(x, dtype=np.float64)
    x2 = x * x
    pw = [x, x2, x2 * x, x2 * x2]
    n = x.shape[0]
    return np.array([math.fsum(v.tolist()) / n for v in pw])


def histogram(x, n_cells, x_lo, x_hi):
    """Counts on the uniform grid of I cells on [x_lo, x_hi] (eq. (binning)).
    Cell i is [x_i, x_{i+1}) with the index floor((x - x_lo) * I/(x_hi - x_lo));
    particles outside the grid are counted in the end cells."""
    x = np.asarray(x, dtype=np.float64)
    inv_h = n_cells / (x_hi - x_lo)
    c = np.floor((x - x_lo) * inv_h)
    c = np.clip(c, 0, n_cells - 1).astype(np.int64)
    return np.bincount(c, minlength=n_cells).astype(np.uint32)


def restrict(x, n_q):
    """R: particle slow coordinates -> (knots, rank, perm, xs)."""
    perm, rank, xs = sort_ranks(x)
    return hazen_knots(xs, n_q), rank, perm, xs
