"""Pins for the oracle's parareal level: the quantile iterator and its
monotone repair (Sec. 4.4), fast-marginal matching (Sec. 5.1) with its
projection property (eq. (projection)), the generic iteration against the
closed form of classical parareal for a linear scalar problem (Sec. 3.1),
and the exactness property of the micro-macro iteration (Sec. 3.3.3)."""
import math
from math import comb

import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as hs
from sklearn.isotonic import IsotonicRegression

from oracle import coarse as C
from oracle import iterate as I
from oracle import particles as P
from oracle import restrict as R


@given(hs.lists(hs.floats(-5, 5, allow_nan=False), min_size=1, max_size=120))
@settings(max_examples=300, deadline=None)
def test_pava_matches_isotonic_regression(v):
    v = np.array(v)
    ours = I.pava(v)
    ref = IsotonicRegression().fit_transform(np.arange(len(v)), v)
    assert np.abs(ours - ref).max() <= 1e-12 * (1 + np.abs(v).max())
    assert np.all(np.diff(ours) >= 0)


def test_pava_pair_average_and_identity():
    assert list(I.pava(np.array([0.0, 2.0, 1.0, 3.0]))) == [0.0, 1.5, 1.5, 3.0]
    v = np.sort(np.random.default_rng(0).standard_normal(101))
    assert np.array_equal(I.pava(v), v)


def test_iterator_property_bitwise():
    rng = np.random.default_rng(1)
    qf = np.sort(rng.standard_normal(101))
    qc = np.sort(rng.standard_normal(101))
    assert np.array_equal(I.j_quantile(qc, qf, qc.copy()), qf)


def test_iterator_shift():
    rng = np.random.default_rng(2)
    qf = np.sort(rng.standard_normal(101))
    qc = np.sort(rng.standard_normal(101))
    out = I.j_quantile(qc + 0.375, qf, qc)
    assert np.abs(out - (qf + 0.375)).max() < 1e-15


def test_match_projection_bitwise():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(5001)
    q, rank, _, _ = R.restrict(x, 100)
    assert np.array_equal(I.match_quantiles(x, rank, q.copy(), q), x)


def test_match_translation_and_scaling():
    rng = np.random.default_rng(4)
    x = rng.standard_normal(4000)
    q, rank, _, xs = R.restrict(x, 100)
    assert np.abs(I.match_quantiles(x, rank, q + 0.25, q) - (x + 0.25)).max() < 1e-14
    # target = affine image of the prior's knots: X = Xbar + delta is the
    # same affine image wherever Xbar's mid-rank level interpolates linearly
    y = I.match_quantiles(x, rank, 2.0 * q, q)
    r = R.restrict(y, 100)[0]
    assert np.abs(r - 2.0 * q)[2:-2].max() < 0.01  # the tail knots move with the extreme particles


def test_match_is_weakly_consistent():
    """R(M(q, Xbar)) is close to q (error O(1/P) plus interpolation)."""
    rng = np.random.default_rng(5)
    x = rng.standard_normal(100_000)
    q, rank, _, _ = R.restrict(x, 100)
    target = np.sort(rng.standard_normal(100_000) * 0.8 + 0.3)
    qt = R.hazen_knots(target, 100)
    y = I.match_quantiles(x, rank, qt, q)
    assert np.abs(R.restrict(y, 100)[0] - qt)[5:-5].max() < 5e-3
    assert np.array_equal(np.argsort(y, kind="stable")[:10], np.argsort(x, kind="stable")[:10])


def test_classical_parareal_closed_form():
    """Generic driver with scalar states, identity restriction/matching and
    the additive iterator: for du/dt = -u with fine F = exp(-dT) and coarse
    G = 1/(1 + dT) per slice, u_k^n = sum_{j<=k} C(n, j) (F - G)^j G^(n-j) u0."""
    K, dT, u0 = 12, 0.3, 1.7
    Fv, Gv = np.exp(-dT), 1.0 / (1.0 + dT)
    pr = I.Parareal(u0, K, fine=lambda n, u: Fv * u, coarse=lambda n, r: Gv * r,
                    restrict=lambda u: u, match=lambda r, prior: r,
                    jump=lambda c, f, cs: c + f - cs)
    for k in range(0, 8):
        for n in range(K + 1):
            ref = sum(comb(n, j) * (Fv - Gv) ** j * Gv ** (n - j) for j in range(min(k, n) + 1)) * u0
            assert abs(pr.u[n] - ref) < 1e-13, (k, n)
        pr.iterate()


def _cfg_small(K=5, n=2000, T=0.25, dt=1e-3, I_cells=60, reuse=False, seed=0):
    s = P.Sde(lam=1.0, eps=0.1, beta=2.0)
    grid = C.Grid(I_cells)
    return I.micmac_parareal(s, seed, 0, n, T, dt, K, grid, 100, reuse_coarse=reuse)


def test_micmac_zeroth_iteration():
    pr, hp = _cfg_small()
    q0 = R.restrict(hp["x0"], 100)[0]
    assert np.array_equal(pr.rho[0], q0)
    for n in range(1, pr.K + 1):
        qn, _ = C.coarse_step(pr.rho[n - 1], hp["E"][n - 1], C.Grid(60))
        assert np.array_equal(pr.rho[n], qn)
        # fast variables untouched by matching, slow ones moved by the knot differences
        assert np.array_equal(pr.u[n].y, hp["y0"])


def test_micmac_exactness_bitwise():
    """After k iterations the states at n <= k equal the serial fine run
    bitwise (projection + eq. (iterator_property)); after K iterations the
    whole trajectory does."""
    for reuse in (False, True):
        pr, hp = _cfg_small(reuse=reuse)
        ref_states, ref_q = I.sequential_reference(hp, pr.K, 100)
        for k in range(1, pr.K + 1):
            pr.iterate()
            for n in range(0, k + 1):
                assert np.array_equal(pr.u[n].x, ref_states[n].x), (reuse, k, n)
                assert np.array_equal(pr.u[n].y, ref_states[n].y), (reuse, k, n)
        for n in range(pr.K + 1):
            assert I.quantile_error(pr.u[n].restricted(100)[0], ref_q[n]) == 0.0


def test_micmac_converges_before_K():
    """The quantile error to the serial run drops with the iterations."""
    pr, hp = _cfg_small(K=8, n=4000, T=0.8)
    _, ref_q = I.sequential_reference(hp, pr.K, 100)

    def err():
        return max(I.quantile_error(pr.u[n].restricted(100)[0], ref_q[n]) for n in range(pr.K + 1))

    e0 = err()
    pr.iterate()
    e1 = err()
    pr.iterate()
    e2 = err()
    assert e1 < e0 and e2 < e1


def test_schedule():
    S, dt = I.total_steps(10.0, 1e-4)
    assert S == 100_000 and dt == 1e-4
    b = I.slice_bounds(S, 64)
    assert b[0] == 0 and b[-1] == S and set(np.diff(b)) == {1562, 1563}
    S, dt = I.total_steps(2.0, 0.0123 / 20)
    assert S == round(2.0 / (0.0123 / 20)) and abs(S * dt - 2.0) < 1e-12


def test_quantile_error_hand_values():
    """The RMS over all Q + 1 knots (Sec. 6's error measure taken on the
    knots): one knot off by 3 among four gives sqrt(9/4) = 1.5 exactly (a mean
    over Q = 3 would give sqrt(3)); a constant offset c gives |c|; the order
    of the arguments does not matter."""
    q = np.array([0.0, 1.0, 2.0, 3.0])
    assert I.quantile_error(q + np.array([3.0, 0.0, 0.0, 0.0]), q) == 1.5
    assert I.quantile_error(q - 0.25, q) == 0.25
    a = np.array([0.5, -1.0, 2.0, 0.0, 4.0])
    b = np.array([0.0, 1.0, 2.0, -2.0, 1.0])
    # differences 0.5, -2, 0, 2, 3: squares sum to 17.25 over 5 knots
    assert I.quantile_error(a, b) == I.quantile_error(b, a) == math.sqrt(17.25 / 5.0)
