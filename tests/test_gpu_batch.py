"""GPU tests of the batched form: many uneven instances in one persistent
launch per phase (optionally a hipGraph), against the same kernels launched
instance by instance (bitwise), against single-instance handles and against
the oracle's iteration for each instance."""
import sys

import numpy as np
import pytest

import paper_1912_09240_amd as pr
from oracle import coarse as OC
from oracle import iterate as OI
from oracle import particles as OP

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
    stream = torch.cuda.Stream()  # graph capture needs a non-default stream
    with torch.cuda.stream(stream):
        yield torch
    torch.cuda.synchronize()


# (eps, lambda, n, K, T): uneven on purpose, incl. a ragged particle count
INSTANCES = [(0.05, 1.3, 3000, 4, 0.2), (0.1, 0.7, 1537, 7, 0.3), (0.02, 1.9, 4096, 3, 0.06),
             (0.08, 1.0, 700, 5, 0.25), (0.03, 0.55, 2049, 6, 0.12)]
CELLS, NQ = 60, 50


def _make(torch, flags=0, inst=INSTANCES, ids=None):
    sdes, scheds, ns = [], [], []
    for eps, lam, n, K, T in inst:
        dt = eps / 20
        S = int(round(T / dt))
        sdes.append(pr.Sde(lam=lam, eps=eps, beta=2.0))
        scheds.append(pr.Schedule(S, K, T / S))
        ns.append(n)
    h = pr.pr_parareal_batch_create(sdes, scheds, ns, pr.Grid(n_cells=CELLS, n_q=NQ), 7,
                                    instances=ids, flags=flags)
    return h


def _states(torch, h, inst=INSTANCES):
    out = []
    for i, (eps, lam, n, K, T) in enumerate(inst):
        for t in range(K + 1):
            x = torch.empty(n, dtype=torch.float64, device="cuda")
            y = torch.empty(n, dtype=torch.float64, device="cuda")
            q = torch.empty(NQ + 1, dtype=torch.float64, device="cuda")
            pr.pr_parareal_batch_state(h, i, t, x=x, y=y, q=q)
            out.append((x, y, q))
    torch.cuda.synchronize()
    return [(a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()) for a, b, c in out]


def test_draw_instances_matches_oracle(torch_dev):
    torch = torch_dev
    _say("draw instances")
    out = torch.empty((256, 4), dtype=torch.float64, device="cuda")
    pr.pr_draw_instances(0, 256, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    for i in range(256):
        eps, lam, n, K = OP.instance_params(0, i)
        assert abs(o[i, 0] - eps) <= 2 * np.spacing(eps) and abs(o[i, 1] - lam) <= 2 * np.spacing(lam)
        assert 2 ** int(o[i, 2]) == n and int(o[i, 3]) == K


def test_launch_modes_bitwise(torch_dev):
    """Batched launches, the captured graph and instance-by-instance launches
    give the same bits; the autotuned shape too."""
    torch = torch_dev
    _say("batch modes")
    results = []
    for mode, flags in ((pr.PR_LAUNCH_PER_INSTANCE, 0), (pr.PR_LAUNCH_BATCHED, 0), (pr.PR_LAUNCH_GRAPH, 0),
                        (pr.PR_LAUNCH_BATCHED, pr.PR_AUTOTUNE), (pr.PR_LAUNCH_GRAPH, pr.PR_REUSE_COARSE)):
        h = _make(torch, flags)
        try:
            pr.pr_parareal_batch_iterate(h, 3, mode)
            results.append((flags, _states(torch, h)))
            if flags & pr.PR_AUTOTUNE:
                info = pr.pr_parareal_batch_info(h)
                assert info["block"] in (128, 256) and info["ppt"] in (1, 2, 4)
                assert info["split_sort"] is False  # no ensemble of 2^16 keys here
        finally:
            pr.pr_parareal_batch_destroy(h)
    ref = results[0][1]
    for flags, st in results[1:4]:
        for (a, b, c), (a0, b0, c0) in zip(st, ref):
            assert np.array_equal(a, a0) and np.array_equal(b, b0) and np.array_equal(c, c0)
    # the reuse variant differs in general but keeps the initial states
    assert np.array_equal(results[4][1][0][0], ref[0][0])


# ensembles the splitter sort takes (2^16 keys and more, one of them ragged)
# beside ones the radix passes sort, in one batch
LARGE_INSTANCES = [(0.05, 1.3, 65536, 3, 0.1), (0.1, 0.7, 3000, 4, 0.2), (0.02, 1.9, 70001, 2, 0.02),
                   (0.08, 1.0, 131072, 3, 0.12), (0.03, 0.55, 4096, 5, 0.06)]


def test_launch_modes_bitwise_with_large_ensembles(torch_dev):
    """A batch whose fine results are sorted in two layouts, the ensembles of
    2^16 keys and more by splitters and buckets (as many buckets as 4096
    keys fill) and the rest by radix passes: batched launches and graph
    replays give the bits of instance-by-instance launches (whose sorts take
    each instance's ensembles alone) over three iterations, states and
    knots; so do the launches with the fine shape and the sort tuned."""
    torch = torch_dev
    _say("batch modes, large ensembles")
    results = []
    for mode, flags in ((pr.PR_LAUNCH_PER_INSTANCE, 0), (pr.PR_LAUNCH_BATCHED, 0), (pr.PR_LAUNCH_GRAPH, 0),
                        (pr.PR_LAUNCH_BATCHED, pr.PR_AUTOTUNE)):
        h = _make(torch, flags, inst=LARGE_INSTANCES)
        try:
            if flags == 0:
                assert pr.pr_parareal_batch_info(h)["split_sort"] is True
            pr.pr_parareal_batch_iterate(h, 3, mode)
            results.append(_states(torch, h, inst=LARGE_INSTANCES))
        finally:
            pr.pr_parareal_batch_destroy(h)
    ref = results[0]
    for st in results[1:]:
        for (a, b, c), (a0, b0, c0) in zip(st, ref):
            assert np.array_equal(a, a0) and np.array_equal(b, b0) and np.array_equal(c, c0)


def test_batch_matches_oracle_per_instance(torch_dev):
    torch = torch_dev
    _say("batch vs oracle")
    inst = INSTANCES[:3]
    h = _make(torch, 0, inst, ids=[11, 3, 40])
    try:
        pr.pr_parareal_batch_iterate(h, 2, pr.PR_LAUNCH_BATCHED)
        st = _states(torch, h, inst)
    finally:
        pr.pr_parareal_batch_destroy(h)
    k = 0
    for (eps, lam, n, K, T), iid in zip(inst, [11, 3, 40]):
        po, _ = OI.micmac_parareal(OP.Sde(lam=lam, eps=eps, beta=2.0), 7, iid, n, T, eps / 20, K, OC.Grid(CELLS), NQ)
        po.iterate()
        po.iterate()
        for t in range(K + 1):
            x, y, q = st[k]
            k += 1
            assert np.abs(q - po.u[t].restricted(NQ)[0]).max() < 1e-10, (iid, t)
            assert np.abs(x - po.u[t].x).max() < 1e-9, (iid, t)
            assert np.abs(y - po.u[t].y[0]).max() < 1e-9, (iid, t)


def test_batch_exactness(torch_dev):
    """After max K iterations every instance equals its serial fine run:
    knot error exactly zero against the GPU's own serial runs."""
    torch = torch_dev
    _say("batch exactness")
    inst = INSTANCES[:3]
    h = _make(torch, 0, inst)
    try:
        pr.pr_parareal_batch_iterate(h, max(K for (_, _, _, K, _) in inst), pr.PR_LAUNCH_GRAPH)
        st = _states(torch, h, inst)
    finally:
        pr.pr_parareal_batch_destroy(h)
    k = 0
    for i, (eps, lam, n, K, T) in enumerate(inst):
        dt = eps / 20
        S = int(round(T / dt))
        sde = pr.Sde(lam=lam, eps=eps, beta=2.0)
        sched = pr.Schedule(S, K, T / S)
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        pr.pr_init_ensemble(sde, 7, i, n, x, y)
        for t in range(K + 1):
            if t > 0:
                pr.pr_fine_propagate(sde, sched, 7, i, n, t - 1, 1, x, y)
            torch.cuda.synchronize()
            assert np.array_equal(st[k][0], x.cpu().numpy()), (i, t)
            k += 1


def test_batch_equals_single_instance_handles_bitwise(torch_dev):
    """Each instance of a batch against its own single-instance driver
    (pr_parareal_create with the same seed and instance word): the batched
    fine launch, segmented sorts, coarse steps, one-block chains and matching
    carry the arithmetic of the single-instance kernels in the same order, so
    knots and states agree bit for bit after three iterations."""
    torch = torch_dev
    _say("batch vs single-instance handles")
    inst = INSTANCES[:3]
    ids = [11, 3, 40]
    h = _make(torch, 0, inst, ids=ids)
    try:
        pr.pr_parareal_batch_iterate(h, 3, pr.PR_LAUNCH_GRAPH)
        st = _states(torch, h, inst)
    finally:
        pr.pr_parareal_batch_destroy(h)
    k = 0
    for (eps, lam, n, K, T), iid in zip(inst, ids):
        dt = eps / 20
        S = int(round(T / dt))
        hs = pr.pr_parareal_create(pr.Sde(lam=lam, eps=eps, beta=2.0), pr.Schedule(S, K, T / S),
                                   pr.Grid(n_cells=CELLS, n_q=NQ), 7, iid, n)
        try:
            pr.pr_parareal_iterate(hs, 3)
            for t in range(K + 1):
                x = torch.empty(n, dtype=torch.float64, device="cuda")
                y = torch.empty(n, dtype=torch.float64, device="cuda")
                q = torch.empty(NQ + 1, dtype=torch.float64, device="cuda")
                pr.pr_parareal_state(hs, t, x=x, y=y, q=q)
                torch.cuda.synchronize()
                a, b, c = st[k]
                k += 1
                assert np.array_equal(c, q.cpu().numpy()), (iid, t)
                assert np.array_equal(a, x.cpu().numpy()), (iid, t)
                assert np.array_equal(b, y.cpu().numpy()), (iid, t)
        finally:
            pr.pr_parareal_destroy(hs)


def test_batched_workload_full_size_first_iteration(torch_dev):
    """The batched workload at its full size (256 instances drawn from seed
    0, 200 cells, 100 levels, creation as the benchmark does it): after one
    iteration replayed from the graph, every instance's state at the end of
    its first slice is the fine propagation of its initial ensemble over that
    slice, bit for bit (Sec. 3.3.3), and the knots of that state are those of
    the single-instance restriction of it."""
    torch = torch_dev
    _say("batched workload full size")
    draw = torch.empty((256, 4), dtype=torch.float64, device="cuda")
    pr.pr_draw_instances(0, 256, draw)
    d = draw.cpu().numpy()
    sdes, scheds, ns = [], [], []
    for eps, lam, lg, K in d:
        dt = eps / 20
        S = int(round(2.0 / dt))
        sdes.append(pr.Sde(lam=float(lam), eps=float(eps), beta=2.0))
        scheds.append(pr.Schedule(S, int(K), 2.0 / S))
        ns.append(2 ** int(lg))
    h = pr.pr_parareal_batch_create(sdes, scheds, ns, pr.Grid(n_cells=200, n_q=100), 0, flags=pr.PR_AUTOTUNE)
    try:
        pr.pr_parareal_batch_iterate(h, 1, pr.PR_LAUNCH_GRAPH)
        for i in range(256):
            n = ns[i]
            x = torch.empty(n, dtype=torch.float64, device="cuda")
            y = torch.empty(n, dtype=torch.float64, device="cuda")
            pr.pr_init_ensemble(sdes[i], 0, i, n, x, y)
            pr.pr_fine_propagate(sdes[i], scheds[i], 0, i, n, 0, 1, x, y)
            xb = torch.empty(n, dtype=torch.float64, device="cuda")
            yb = torch.empty(n, dtype=torch.float64, device="cuda")
            qb = torch.empty(101, dtype=torch.float64, device="cuda")
            pr.pr_parareal_batch_state(h, i, 1, x=xb, y=yb, q=qb)
            q = torch.empty(101, dtype=torch.float64, device="cuda")
            ws = torch.empty(pr.pr_restrict_workspace_size(n, 1), dtype=torch.uint8, device="cuda")
            pr.pr_restrict_quantiles(x, pr.PR_F64, n, 1, 100, q, ws)
            torch.cuda.synchronize()
            assert torch.equal(xb, x) and torch.equal(yb, y), i
            assert torch.equal(qb, q), i
    finally:
        pr.pr_parareal_batch_destroy(h)


def test_batched_workload_flagged_ensembles_sorted_alone(torch_dev):
    """The full-size batched workload over three iterations (one in batched
    launches, two graph replays) against the same three iterations instance
    by instance: the knots of every state of every instance agree bit for
    bit.  In these iterations the matched-knot kernels cannot isolate some
    order statistics of a few new states; only the ensembles so flagged are
    sorted (fewer than all of them), and their knots still agree."""
    torch = torch_dev
    _say("batched workload flagged ensembles")
    draw = torch.empty((256, 4), dtype=torch.float64, device="cuda")
    pr.pr_draw_instances(0, 256, draw)
    d = draw.cpu().numpy()
    sdes, scheds, ns = [], [], []
    for eps, lam, lg, K in d:
        dt = eps / 20
        S = int(round(2.0 / dt))
        sdes.append(pr.Sde(lam=float(lam), eps=float(eps), beta=2.0))
        scheds.append(pr.Schedule(S, int(K), 2.0 / S))
        ns.append(2 ** int(lg))
    grid = pr.Grid(n_cells=200, n_q=100)
    rows = sum(sc.n_slices + 1 for sc in scheds)
    segments = sum(sc.n_slices for sc in scheds)

    def knots(h):
        out = torch.empty((rows, 101), dtype=torch.float64, device="cuda")
        r = 0
        for i, sc in enumerate(scheds):
            for t in range(sc.n_slices + 1):
                pr.pr_parareal_batch_state(h, i, t, q=out[r])
                r += 1
        torch.cuda.synchronize()
        return out.cpu()

    stream = torch.cuda.Stream()  # graph capture needs a non-default stream
    with torch.cuda.stream(stream):
        h = pr.pr_parareal_batch_create(sdes, scheds, ns, grid, 0, flags=pr.PR_AUTOTUNE)
        try:
            info = pr.pr_parareal_batch_info(h)
            pr.pr_parareal_batch_iterate(h, 1, pr.PR_LAUNCH_BATCHED)
            pr.pr_parareal_batch_iterate(h, 2, pr.PR_LAUNCH_GRAPH)
            sorts, sorted_segs = pr.pr_parareal_batch_knot_sorts(h)
            qa = knots(h)
        finally:
            pr.pr_parareal_batch_destroy(h)
        _say(f"  knot sorts {sorts}, ensembles sorted {sorted_segs} of {segments} per iteration, "
             f"fine results sorted by splitters: {info['split_sort']}")
        h = pr.pr_parareal_batch_create(sdes, scheds, ns, grid, 0)
        try:
            pr.pr_parareal_batch_iterate(h, 3, pr.PR_LAUNCH_PER_INSTANCE)
            qb = knots(h)
        finally:
            pr.pr_parareal_batch_destroy(h)
    assert torch.equal(qa, qb)
    assert sorts >= 1, "no flagged ensemble in these iterations: the per-ensemble sort was not exercised"
    assert 0 < sorted_segs < sorts * segments
