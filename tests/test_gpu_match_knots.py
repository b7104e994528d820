"""GPU parity of the knots of matched ensembles taken without a sort
(pr_match_knots) against the sort of the matched ensembles
(pr_restrict_quantiles), bit for bit, through the C ABI; the sort's knots are
themselves pinned to the oracle by the restriction tests.  Also: the flag is
raised where the matched values are far from the prior's order, and the
parareal driver takes its knots this way on the workloads."""
import sys

import numpy as np
import pytest

import paper_1912_09240_amd as pr
from oracle import iterate as OI
from oracle import restrict as OR
from tests import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert pr.available(), "libpr.so not built"
    return torch


def _knots_both_ways(torch, xs_np, nq, shift, precision=pr.PR_F64):
    """Restrict the priors, match them to the prior knots moved by shift(levels)
    and return (knots without a sort, flag, knots of a sort of the matched
    ensembles)."""
    k, n = xs_np.shape
    dt = torch.float64 if precision == pr.PR_F64 else torch.float32
    x = torch.from_numpy(xs_np).to(dt).cuda()
    ws = torch.empty(pr.pr_restrict_workspace_size(n, k, precision), dtype=torch.uint8, device="cuda")
    qp = torch.empty((k, nq + 1), dtype=torch.float64, device="cuda")
    rank = torch.empty((k, n), dtype=torch.int32, device="cuda")
    pr.pr_restrict_quantiles(x, precision, n, k, nq, qp, ws, rank=rank)
    lev = torch.arange(nq + 1, dtype=torch.float64, device="cuda") / nq
    qt = (qp + shift(lev)).contiguous()
    xm = torch.empty_like(x)
    pr.pr_match_quantiles(qt, qp, rank, n, k, nq, x, xm, precision)
    q_fast = torch.full((k, nq + 1), float("nan"), dtype=torch.float64, device="cuda")
    flag = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    pr.pr_match_knots(qt, qp, n, k, nq, ws, q_fast, flag, precision)
    torch.cuda.synchronize()
    fl = int(flag.item())
    q_sort = torch.empty((k, nq + 1), dtype=torch.float64, device="cuda")
    ws2 = torch.empty_like(ws)
    pr.pr_restrict_quantiles(xm, precision, n, k, nq, q_sort, ws2)
    torch.cuda.synchronize()
    return q_fast.cpu().numpy(), fl, q_sort.cpu().numpy()


def _smooth(lev):
    return 0.01 + 0.02 * (3.0 * 3.141592653589793 * lev).sin()


@pytest.mark.parametrize("k,n,ties", [(1, 2, True), (3, 63, True), (2, 64, True), (2, 65, True), (4, 1000, True),
                                      (3, 4096, True), (2, 4097, True), (5, 70_001, False), (5, 70_001, True),
                                      (2, 2 ** 20, False)])
def test_match_knots_equal_sorted_knots(torch_dev, k, n, ties):
    """Continuous priors always give the knots without a sort.  With the
    inputs' exact ties, a run of hundreds of equal priors (the signed zeros at
    the larger sizes) becomes a monotone run of matched values that may
    overlap its neighbours for more than 64 ranks: then the flag may be
    raised; where it is not, the knots are still exact."""
    _say(f"match knots k={k} n={n} ties={ties}")
    xs = inputs.slow_values(300 + n, k, n, ties=ties)
    qf, fl, qs = _knots_both_ways(torch_dev, xs, 100, _smooth)
    if not ties or n <= 5000:
        assert fl == 0
    if fl == 0:
        assert np.array_equal(qf.view(np.uint64), qs.view(np.uint64))


@pytest.mark.parametrize("k,n", [(3, 5_000), (2, 70_001)])
def test_match_knots_against_the_oracle(torch_dev, k, n):
    """The knots without a sort against the oracle's own chain: its
    restriction of the priors, its matching to the moved knots, its sort and
    Hazen knots of the matched ensembles -- bit for bit."""
    torch = torch_dev
    _say(f"match knots vs oracle k={k} n={n}")
    nq = 100
    xs = inputs.slow_values(900 + n, k, n, ties=False)
    lev = np.arange(nq + 1) / nq
    shift = 0.01 + 0.02 * np.sin(3.0 * np.pi * lev)
    qp_o, qt_o, qref = [], [], []
    for s in range(k):
        _, rank, srt = OR.sort_ranks(xs[s])
        qp = OR.hazen_knots(srt, nq)
        qt = qp + shift
        xm = OI.match_quantiles(xs[s], rank, qt, qp)
        qp_o.append(qp)
        qt_o.append(qt)
        qref.append(OR.hazen_knots(OR.sort_ranks(xm)[2], nq))
    x = torch.from_numpy(xs).cuda()
    ws = torch.empty(pr.pr_restrict_workspace_size(n, k), dtype=torch.uint8, device="cuda")
    qp = torch.empty((k, nq + 1), dtype=torch.float64, device="cuda")
    rank = torch.empty((k, n), dtype=torch.int32, device="cuda")
    pr.pr_restrict_quantiles(x, pr.PR_F64, n, k, nq, qp, ws, rank=rank)
    torch.cuda.synchronize()
    assert np.array_equal(qp.cpu().numpy(), np.stack(qp_o))
    qt = torch.from_numpy(np.stack(qt_o)).cuda()
    q = torch.empty((k, nq + 1), dtype=torch.float64, device="cuda")
    flag = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    pr.pr_match_knots(qt, qp, n, k, nq, ws, q, flag)
    torch.cuda.synchronize()
    assert int(flag.item()) == 0
    assert np.array_equal(q.cpu().numpy().view(np.uint64), np.stack(qref).view(np.uint64))


@pytest.mark.parametrize("nq", [1, 7, 100, 1000])
def test_match_knots_levels(torch_dev, nq):
    _say(f"match knots nq={nq}")
    xs = inputs.slow_values(41 + nq, 3, 20_000, ties=False)
    qf, fl, qs = _knots_both_ways(torch_dev, xs, nq, _smooth)
    assert fl == 0
    assert np.array_equal(qf.view(np.uint64), qs.view(np.uint64))


def test_match_knots_ties_and_identity(torch_dev):
    """Values on a coarse lattice (runs of thousands of equal keys).  With
    unchanged knots the matched ensembles are the priors; with knots moved by
    an increasing function of the level every run of equal priors becomes an
    increasing run below the next one, so every position is a cut; with a
    decreasing one every run becomes a strictly decreasing run of thousands
    of ranks, no position inside it is a cut, and the flag is raised."""
    torch = torch_dev
    _say("match knots ties")
    rng = np.random.default_rng(8)
    xs = np.ascontiguousarray(np.round(rng.normal(0.0, 1.0, (3, 50_000)) * 4.0) / 4.0)
    qf, fl, qs = _knots_both_ways(torch, xs, 100, lambda lev: 0.0 * lev)
    assert fl == 0 and np.array_equal(qf.view(np.uint64), qs.view(np.uint64))
    qf, fl, qs = _knots_both_ways(torch, xs, 100, lambda lev: 0.05 * lev)
    assert fl == 0 and np.array_equal(qf.view(np.uint64), qs.view(np.uint64))
    _, fl, _ = _knots_both_ways(torch, xs, 100, lambda lev: -0.05 * lev)
    assert fl == 1


def test_match_knots_fp32(torch_dev):
    _say("match knots fp32")
    xs = inputs.slow_values(77, 3, 30_001, ties=False)
    qf, fl, qs = _knots_both_ways(torch_dev, xs, 100, _smooth, precision=pr.PR_F32)
    assert fl == 0
    assert np.array_equal(qf.view(np.uint64), qs.view(np.uint64))


def test_match_knots_flag_far_from_prior_order(torch_dev):
    """Targets that collapse the ensemble onto one value scramble the prior's
    order: the order statistics cannot be isolated and the flag says so."""
    _say("match knots flag")
    xs = inputs.slow_values(5, 2, 100_000, ties=False)
    torch = torch_dev
    k, n, nq = 2, 100_000, 100
    x = torch.from_numpy(xs).cuda()
    ws = torch.empty(pr.pr_restrict_workspace_size(n, k), dtype=torch.uint8, device="cuda")
    qp = torch.empty((k, nq + 1), dtype=torch.float64, device="cuda")
    rank = torch.empty((k, n), dtype=torch.int32, device="cuda")
    pr.pr_restrict_quantiles(x, pr.PR_F64, n, k, nq, qp, ws, rank=rank)
    qt = torch.full_like(qp, 0.5)
    q = torch.empty_like(qp)
    flag = torch.zeros((1,), dtype=torch.int32, device="cuda")
    pr.pr_match_knots(qt, qp, n, k, nq, ws, q, flag)
    torch.cuda.synchronize()
    assert int(flag.item()) == 1


def test_parareal_takes_knots_without_sort(torch_dev):
    """On the small workload every iteration's new knots come from the fine
    results' sort (no sort of the new states), and the knots agree with the
    sort of the states."""
    torch = torch_dev
    cfg = inputs.CFG_SMALL
    _say("parareal knots without sort")
    S = int(round(cfg["T"] / cfg["dt"]))
    h = pr.pr_parareal_create(pr.Sde(lam=cfg["lam"], eps=cfg["eps"], beta=cfg["beta"]),
                              pr.Schedule(S, cfg["K"], cfg["T"] / S), pr.Grid(n_cells=cfg["cells"], n_q=cfg["nq"]),
                              0, 0, cfg["n"], 0)
    try:
        n, nq = cfg["n"], cfg["nq"]
        ws = torch.empty(pr.pr_restrict_workspace_size(n, 1), dtype=torch.uint8, device="cuda")
        for _ in range(3):
            pr.pr_parareal_iterate(h, 1)
            for t in range(cfg["K"] + 1):
                x = torch.empty(n, dtype=torch.float64, device="cuda")
                q = torch.empty(nq + 1, dtype=torch.float64, device="cuda")
                qs = torch.empty(nq + 1, dtype=torch.float64, device="cuda")
                pr.pr_parareal_state(h, t, x=x, q=q)
                pr.pr_restrict_quantiles(x, pr.PR_F64, n, 1, nq, qs, ws)
                torch.cuda.synchronize()
                assert torch.equal(q, qs), t
        assert pr.pr_parareal_knot_sorts(h) == 0
    finally:
        pr.pr_parareal_destroy(h)


def test_parareal_sorts_new_states_when_needed(torch_dev):
    """With three particles in each of 32 slices the workspace has no room
    for the chunk extremes: every iteration then takes the new knots by a
    sort of the new states, and they still equal the sort of the states."""
    torch = torch_dev
    _say("parareal knots by sort")
    n, K, nq = 3, 32, 10
    h = pr.pr_parareal_create(pr.Sde(lam=1.0, eps=0.1, beta=2.0), pr.Schedule(320, K, 1e-3),
                              pr.Grid(n_cells=50, n_q=nq), 0, 0, n, 0)
    try:
        ws = torch.empty(pr.pr_restrict_workspace_size(n, 1), dtype=torch.uint8, device="cuda")
        for _ in range(2):
            pr.pr_parareal_iterate(h, 1)
        for t in range(K + 1):
            x = torch.empty(n, dtype=torch.float64, device="cuda")
            q = torch.empty(nq + 1, dtype=torch.float64, device="cuda")
            qs = torch.empty(nq + 1, dtype=torch.float64, device="cuda")
            pr.pr_parareal_state(h, t, x=x, q=q)
            pr.pr_restrict_quantiles(x, pr.PR_F64, n, 1, nq, qs, ws)
            torch.cuda.synchronize()
            assert torch.equal(q, qs), t
        assert pr.pr_parareal_knot_sorts(h) == 2
    finally:
        pr.pr_parareal_destroy(h)


def test_parareal_fp32_knots_and_exactness(torch_dev):
    """FP32 stepping in the driver: the new knots come from the fine results'
    32-bit sort without a second sort and equal the sort of the states, and
    after K iterations every state is the serial FP32 fine run bit for bit."""
    torch = torch_dev
    _say("parareal fp32")
    n, K, nq, S = 5000, 6, 50, 600
    sde = pr.Sde(lam=1.0, eps=0.1, beta=2.0, precision=pr.PR_F32)
    sched = pr.Schedule(S, K, 1e-3)
    h = pr.pr_parareal_create(sde, sched, pr.Grid(n_cells=100, n_q=nq), 0, 0, n, 0)
    try:
        x = torch.empty(n, dtype=torch.float32, device="cuda")
        y = torch.empty(n, dtype=torch.float32, device="cuda")
        pr.pr_init_ensemble(sde, 0, 0, n, x, y)
        ref = [x.clone()]
        for s in range(K):
            pr.pr_fine_propagate(sde, sched, 0, 0, n, s, 1, x, y)
            ref.append(x.clone())
        ws = torch.empty(pr.pr_restrict_workspace_size(n, 1, pr.PR_F32), dtype=torch.uint8, device="cuda")
        for k in range(1, K + 1):
            pr.pr_parareal_iterate(h, 1)
            for t in range(K + 1):
                xs = torch.empty(n, dtype=torch.float32, device="cuda")
                q = torch.empty(nq + 1, dtype=torch.float64, device="cuda")
                qs = torch.empty(nq + 1, dtype=torch.float64, device="cuda")
                pr.pr_parareal_state(h, t, x=xs, q=q)
                pr.pr_restrict_quantiles(xs, pr.PR_F32, n, 1, nq, qs, ws)
                torch.cuda.synchronize()
                assert torch.equal(q, qs), (k, t)
                if t <= k:
                    assert torch.equal(xs, ref[t]), (k, t)
        assert pr.pr_parareal_knot_sorts(h) == 0
    finally:
        pr.pr_parareal_destroy(h)
