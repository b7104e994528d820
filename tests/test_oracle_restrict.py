"""Pins for the oracle's restriction (Sec. 3.2.2 and Sec. 4.4): the
orderable key, the stable order by (value, index), the midpoint (Hazen)
quantile knots against numpy's own implementation, moments against exact
rational sums, histogram against a brute-force loop."""
import math
from fractions import Fraction

import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as hs

from oracle import restrict as R

finite = hs.floats(allow_nan=False, allow_infinity=True, width=64)


@given(hs.lists(finite, min_size=1, max_size=60))
@settings(max_examples=300, deadline=None)
def test_key_order_is_numeric_order(vals):
    x = np.array(vals, dtype=np.float64)
    k = R.orderable_key(x)
    for i in range(len(x)):
        for j in range(len(x)):
            if x[i] < x[j]:
                assert k[i] < k[j]
            if x[i] == x[j] and np.signbit(x[i]) == np.signbit(x[j]):
                assert k[i] == k[j]


def test_negative_zero_orders_first():
    k = R.orderable_key(np.array([0.0, -0.0]))
    assert k[1] < k[0]


@given(hs.lists(hs.sampled_from([-2.5, -1.0, -0.0, 0.0, 0.5, 1.0, 3.25]) | finite, min_size=1, max_size=80))
@settings(max_examples=300, deadline=None)
def test_sort_is_stable_brute_force(vals):
    x = np.array(vals, dtype=np.float64)
    perm, rank, xs = R.sort_ranks(x)
    # brute force: order by (value, sign of zero, index)
    ref = sorted(range(len(x)), key=lambda i: (x[i], 0 if (x[i] == 0 and math.copysign(1, x[i]) < 0) else 1, i))
    assert list(perm) == ref
    assert np.array_equal(rank[perm], np.arange(len(x)))
    assert np.array_equal(xs.view(np.uint64), x[perm].view(np.uint64))


def test_hazen_matches_numpy():
    rng = np.random.default_rng(0)
    for N in (1, 2, 3, 7, 100, 101, 1000, 4097):
        x = rng.standard_normal(N)
        xs = np.sort(x)
        for Q in (1, 2, 10, 100):
            q = R.hazen_knots(xs, Q)
            ref = np.quantile(x, np.arange(Q + 1) / Q, method="hazen")
            # interpolation between two order statistics: a few ulp of their
            # magnitude, plus numpy's rounding of p = j/Q before scaling by N
            # (an error of N eps in the position times the local gap)
            gap = np.diff(xs).max() if N > 1 else 0.0
            tol = 4 * np.spacing(np.abs(x).max()) + N * 2.3e-16 * gap
            assert np.all(np.abs(q - ref) <= tol), (N, Q)
            assert np.all(np.diff(q) >= 0)


def test_hazen_definition_cases():
    xs = np.array([0.0, 1.0, 2.0, 4.0])  # N = 4
    q = R.hazen_knots(xs, 4)  # p = 0, .25, .5, .75, 1 -> t = -.5, .5, 1.5, 2.5, 3.5
    assert list(q) == [0.0, 0.5, 1.5, 3.0, 4.0]
    q = R.hazen_knots(xs, 2)  # p = .5: t = 1.5 -> midpoint of 1 and 2
    assert list(q) == [0.0, 1.5, 4.0]


def test_hazen_monotone_on_near_ties():
    base = 1.0
    xs = np.array([base, np.nextafter(base, 2), np.nextafter(np.nextafter(base, 2), 2)] * 1)
    xs = np.sort(np.concatenate([xs, xs + 1e-300]))
    q = R.hazen_knots(xs, 97)
    assert np.all(np.diff(q) >= 0)


def test_moments_exact():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(2000) * 3
    mom = R.moments(x)
    for m in range(1, 5):
        terms = [x * x, x * x * x, (x * x) * (x * x)]
        v = x if m == 1 else terms[m - 2]
        exact = sum(Fraction(float(t)) for t in v) / len(x)
        assert abs(mom[m - 1] - float(exact)) <= 2 * np.spacing(abs(float(exact))) + 1e-300


def test_histogram_brute_force():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.standard_normal(5000) * 1.5, [-3.0, 3.0, -10, 10, 2.97, -2.9999999]])
    I, lo, hi = 200, -3.0, 3.0
    h = R.histogram(x, I, lo, hi)
    ref = np.zeros(I, dtype=np.int64)
    inv = I / (hi - lo)
    for v in x:
        c = math.floor((v - lo) * inv)
        ref[min(max(c, 0), I - 1)] += 1
    assert np.array_equal(h, ref)
    assert h.sum() == len(x)


def test_hazen_at_equals_the_knots_at_their_levels():
    """The single-level quantile of the observables at p = j/Q is the knot j
    of the same sample (Sec. 4.4 rules), ends included: bit for bit where
    j/Q is exact in binary (Q a power of two), else within the rounding of
    the level p = j/Q (N eps in the position times the local gap)."""
    rng = np.random.default_rng(3)
    for N in (1, 2, 5, 64, 1001):
        xs = np.sort(rng.standard_normal(N))
        gap = np.diff(xs).max() if N > 1 else 0.0
        for Q in (1, 4, 10, 64, 100, 128):
            q = R.hazen_knots(xs, Q)
            exact = Q & (Q - 1) == 0
            for j in range(Q + 1):
                v = R.hazen_at(xs, j / Q)[0]
                if exact:
                    assert v == q[j], (N, Q, j)
                else:
                    assert abs(v - q[j]) <= 2 * np.spacing(np.abs(xs).max()) + N * 2.3e-16 * gap, (N, Q, j)


def test_hazen_at_matches_numpy_at_arbitrary_levels():
    """numpy's own midpoint quantile at levels that are not knot levels,
    the clamped ends and the interpolation position returned with it."""
    rng = np.random.default_rng(4)
    for N in (1, 2, 3, 17, 500, 4097):
        x = rng.standard_normal(N) * 2.0
        xs = np.sort(x)
        gap = np.diff(xs).max() if N > 1 else 0.0
        for p in np.concatenate([[0.0, 1.0, 0.5 / N, 1.0 - 0.5 / N], rng.random(40)]):
            v, r, f = R.hazen_at(xs, float(p))
            ref = np.quantile(x, p, method="hazen")
            tol = 4 * np.spacing(np.abs(x).max()) + N * 2.3e-16 * gap
            assert abs(v - ref) <= tol, (N, p)
            t = p * N - 0.5
            if t <= 0.0:
                assert (v, r, f) == (xs[0], 0, 0.0)
            elif t >= N - 1:
                assert (v, r, f) == (xs[-1], N - 1, 0.0)
            else:
                assert r == math.floor(t) and 0.0 <= f < 1.0 and xs[r] <= v <= xs[r + 1]


def test_hazen_at_worked_example():
    xs = np.array([0.0, 1.0, 2.0, 4.0])  # t = 4p - 1/2
    assert R.hazen_at(xs, 0.1)[0] == 0.0          # t = -0.1: the minimum
    assert R.hazen_at(xs, 0.5)[0] == 1.5          # t = 1.5: midpoint of 1 and 2
    assert R.hazen_at(xs, 0.75)[0] == 3.0         # t = 2.5: midpoint of 2 and 4
    assert R.hazen_at(xs, 0.8125)[0] == 3.5       # t = 2.75: three quarters from 2 to 4
    assert R.hazen_at(xs, 0.95)[0] == 4.0         # t = 3.3: the maximum
