"""Pins of the histogram-state oracle (iterators of Sec. 4, matchings of
Sec. 5) against exact arithmetic, closed forms, geometric properties and
brute force, each chosen so that a plausible slip in the oracle fails one."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import coarse as OC
from oracle import histogram as H
from oracle import iterate as OI
from oracle import particles as OP


def _rand_hist(rng, I, zeros=()):
    r = rng.random(I) + 0.05
    for z in zeros:
        r[z] = 0.0
    return r / r.sum()


def test_restrict_is_the_exact_sum_rounded_once():
    g = OC.Grid(16, -2.0, 2.0)
    rng = np.random.default_rng(1)
    x = rng.normal(0.0, 1.0, 3000)
    x[:5] = [-5.0, 5.0, -2.0, 2.0, 0.0]  # outside, ends, an edge
    w = rng.random(3000) * 1e-3
    rho = H.hist_restrict(x, w, g)
    h = 4.0 / 16
    for i in range(16):
        lo, hi = -2.0 + i * h, -2.0 + (i + 1) * h
        inside = [(xv >= lo or i == 0) and (xv < hi or i == 15) for xv in x]
        exact = sum((Fraction(float(v)) for v, s in zip(w, inside) if s), Fraction(0))
        assert rho[i] == float(exact)
    # equal weights: count * fl(1/P) rounded once
    we = H.equal_weights(3000)
    rho = H.hist_restrict(x, we, g)
    cnt = np.bincount(H.cell_index(x, g), minlength=16)
    assert np.array_equal(rho, np.array([float(Fraction(int(c)) * Fraction(we[0])) for c in cnt]))


def test_quantile_closed_forms_and_support_rules():
    g = OC.Grid(10, 0.0, 10.0)
    uni = np.full(10, 0.1)
    c = H.cdf_edges(uni)
    for p in (0.0, 0.05, 0.31, 0.5, 0.99):
        assert abs(H.quantile_at(uni, c, g, p) - 10.0 * p) < 1e-13
    assert H.quantile_at(uni, c, g, c[-1]) == 10.0
    # support [2, 7): q(0) = 2, q(M) = 7
    r = np.zeros(10)
    r[2:7] = 0.2
    c = H.cdf_edges(r)
    assert H.quantile_at(r, c, g, 0.0) == 2.0 and H.quantile_at(r, c, g, c[-1]) == 7.0
    # a gap [4, 8) between two blocks: the level of the gap maps to its midpoint
    r = np.zeros(10)
    r[[1, 2, 3]] = 0.2
    r[[8, 9]] = 0.2
    c = H.cdf_edges(r)
    assert H.quantile_at(r, c, g, c[4]) == 6.0


def test_quantile_against_dense_inversion():
    g = OC.Grid(12, -1.0, 2.0)
    rng = np.random.default_rng(3)
    r = _rand_hist(rng, 12, zeros=(0, 5, 6, 11))
    c = H.cdf_edges(r)
    xs = np.linspace(-1.0, 2.0, 120001)
    cx = np.interp(xs, g.edges, c)  # the piecewise-linear cdf, sampled densely
    for p in rng.random(40) * c[-1]:
        sel = xs[np.abs(cx - p) <= 1e-12]
        if len(sel) == 0:
            k = np.searchsorted(cx, p)
            sel = xs[k - 1:k + 1]
        mid = 0.5 * (sel.min() + sel.max())
        assert abs(H.quantile_at(r, c, g, p) - mid) < 3e-5


@pytest.mark.parametrize("kind", [H.J_ADD, H.J_MULT, H.J_ROT, H.J_QUANTILE])
def test_iterator_property(kind):
    """J(a, f, a) = f (eq. (iterator_property)): bitwise for the additive and
    multiplicative iterators, to rounding for the others."""
    g = OC.Grid(30, -3.0, 3.0)
    rng = np.random.default_rng(kind)
    a = _rand_hist(rng, 30)
    f = _rand_hist(rng, 30, zeros=(0, 29))
    r = H.jump(kind, a, f, a, g)
    if kind in (H.J_ADD, H.J_MULT):
        assert np.array_equal(r, f)
    else:
        assert np.abs(r - f).max() < 1e-15


def test_additive_hand_example():
    g = OC.Grid(4)
    rc = np.array([0.1, 0.2, 0.3, 0.4])
    rcs = np.array([0.4, 0.3, 0.2, 0.1])
    rf = np.array([0.25, 0.25, 0.25, 0.25])
    # rf + rc - rcs = (-0.05, 0.15, 0.35, 0.55): clip, then scale 1/1.05
    r = H.jump(H.J_ADD, rc, rf, rcs, g)
    assert np.allclose(r, np.array([0.0, 0.15, 0.35, 0.55]) / 1.05, rtol=0, atol=4e-16)
    assert np.all(r >= 0)


def test_multiplicative_hand_example_and_support():
    g = OC.Grid(4)
    rc = np.array([0.1, 0.2, 0.3, 0.4])
    rcs = np.array([0.2, 0.0, 0.4, 0.4])
    rf = np.array([0.3, 0.2, 0.2, 0.3])
    raw = np.array([0.3 * 0.5, 0.0, 0.2 * 0.75, 0.3 * 1.0])
    r = H.jump(H.J_MULT, rc, rf, rcs, g)
    assert np.allclose(r, raw / raw.sum(), rtol=0, atol=4e-16)


def test_rotation_is_a_rotation():
    g = OC.Grid(40)
    rng = np.random.default_rng(7)
    rc = _rand_hist(rng, 40)
    rcs = _rand_hist(rng, 40)
    rf = _rand_hist(rng, 40)
    r = H.jump(H.J_ROT, rc, rf, rcs, g)
    assert np.all(r >= 0) and abs(r.sum() - 1.0) < 1e-14  # norm of sqrt is kept
    # it takes sqrt(rcs) to sqrt(rc)
    assert np.abs(H.jump(H.J_ROT, rc, rcs, rcs, g) - rc).max() < 1e-15
    # and leaves a vector orthogonal to both alone
    rc2, rcs2, rf2 = np.zeros(40), np.zeros(40), np.zeros(40)
    rc2[:10], rcs2[5:20], rf2[25:] = 0.1, 1 / 15, 1 / 15
    assert np.abs(H.jump(H.J_ROT, rc2, rf2, rcs2, g) - rf2).max() < 1e-16


def test_quantile_iterator_corrects_a_shift_exactly():
    """If the two coarse results differ by a translation of m cells, the
    quantile iterator translates the fine result by the same m cells."""
    g = OC.Grid(40, 0.0, 40.0)
    rng = np.random.default_rng(11)
    rcs = np.zeros(40)
    rcs[5:15] = _rand_hist(rng, 10)
    rf = np.zeros(40)
    rf[8:20] = _rand_hist(rng, 12)
    m = 7
    rc = np.roll(rcs, m)
    r = H.jump(H.J_QUANTILE, rc, rf, rcs, g)
    assert np.abs(r - np.roll(rf, m)).max() < 1e-14
    assert abs(r.sum() - 1.0) < 1e-14


def test_marginal_matching_identity_order_and_weak_consistency():
    g = OC.Grid(24)
    rng = np.random.default_rng(5)
    x = rng.normal(0.0, 0.8, 4000)
    w = H.equal_weights(4000)
    rp = H.hist_restrict(x, w, g)
    xn = H.match_marginal(rp, rp, x, g)
    inside = np.abs(x) < 3.0
    assert np.abs(xn - x)[inside].max() < 1e-13
    rt = _rand_hist(rng, 24)
    xn = H.match_marginal(rt, rp, x, g)
    o = np.argsort(x, kind="stable")
    assert np.all(np.diff(xn[o]) >= 0)  # monotone transport
    got = H.hist_restrict(xn, w, g)
    assert np.abs(got - rt).max() <= rp.max() + 1.0 / 4000


def test_unsupported_mass_moves_to_neighbours():
    rp = np.array([0.0, 0.5, 0.0, 0.0, 0.5, 0.0])
    rt = np.array([0.1, 0.2, 0.1, 0.2, 0.3, 0.1])
    r = H.move_unsupported(rt, rp)
    # cell 0: all to cell 1; cells 2, 3: half to 1, half to 4; cell 5: all to 4
    assert np.allclose(r, [0.0, 0.2 + 0.1 + 0.05 + 0.1, 0.0, 0.0, 0.3 + 0.05 + 0.1 + 0.1, 0.0], atol=1e-16)
    assert abs(r.sum() - rt.sum()) < 4e-16


def test_reweighting_reproduces_the_target():
    g = OC.Grid(20)
    rng = np.random.default_rng(9)
    x = rng.normal(0.0, 0.6, 3000)
    w = H.equal_weights(3000)
    rp = H.hist_restrict(x, w, g)
    rt = _rand_hist(rng, 20)
    wn = H.reweight(rt, rp, x, w, g)
    assert np.abs(H.hist_restrict(x, wn, g) - H.move_unsupported(rt, rp)).max() < 1e-15
    assert np.array_equal(H.reweight(rp, rp, x, w, g), w)


@pytest.mark.parametrize("det", [False, True])
def test_resampling_counts(det):
    rng = np.random.default_rng(13)
    P = 2000
    w = rng.random(P) ** 3
    w[::17] = 0.0
    w = w / w.sum()
    slots = H.resample_slots(w, 5, 2, 7, det)
    assert np.all(np.diff(slots) >= 0)  # stratified: slots in particle order
    n = np.bincount(slots, minlength=P)
    q = H.fixed_weights(w)
    T = sum(q)
    expect = [Fraction(v * P, T) for v in q]
    dev = [abs(Fraction(int(a)) - e) for a, e in zip(n, expect)]
    assert max(dev) < (1 if det else 2)  # systematic: floor or ceil; stratified: within 2
    assert np.all(n[::17] == 0)
    # equal weights: the identity, random or deterministic
    assert np.array_equal(H.resample_slots(H.equal_weights(997), 5, 2, 7, det), np.arange(997))


def test_stratified_resampling_is_unbiased():
    P = 50
    w = np.linspace(1.0, 3.0, P)
    w = w / w.sum()
    tot = np.zeros(P)
    reps = 400
    for s in range(reps):
        tot += np.bincount(H.resample_slots(w, s, 0, 0, False), minlength=P)
    mean = tot / reps
    # each count is within 2 of P w, so the standard error is below 1/sqrt(reps)
    assert np.abs(mean - P * w).max() < 4.0 / np.sqrt(reps)


@pytest.mark.parametrize("it", [H.J_ADD, H.J_MULT, H.J_ROT, H.J_QUANTILE])
@pytest.mark.parametrize("mt", [H.M_MARGINAL, H.M_REWEIGHT, H.M_RESAMPLE, H.M_RESAMPLE_DET])
def test_hist_parareal_exactness(oracle_lib, it, mt):
    """After N iterations the states equal the serial fine run (Sec. 3.3.3):
    bitwise when the iterator and the matching keep their fixed points
    exactly, to rounding otherwise.  The grid is chosen so that the fine
    histograms have no empty interior cells: across an empty interior cell
    the union-of-levels quantile iterator interpolates a jump of the
    quantile function linearly and moves mass into the gap, so its iterator
    property holds only for gap-free histograms."""
    sde = OP.Sde(lam=1.0, eps=0.1, beta=2.0)
    g = OC.Grid(20, -2.0, 2.0)
    K = 3
    pr, hp = H.micmac_parareal_hist(sde, 3, 0, 2000, 0.3, 1e-2, K, g, it, mt)
    states, ref = H.sequential_reference_hist(hp, K, g)
    first = []
    for k in range(K):
        pr.iterate()
        first.append(max(H.hist_error(pr.u[n].rho(g), ref[n]) for n in range(K + 1)))
    bitwise = it in (H.J_ADD, H.J_MULT) and mt != H.M_MARGINAL
    for n in range(K + 1):
        if bitwise:
            assert np.array_equal(pr.u[n].x, states[n].x)
        else:
            assert np.abs(pr.u[n].x - states[n].x).max() < 1e-12
    assert first[-1] < 1e-14
