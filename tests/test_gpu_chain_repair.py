"""GPU parity of the quantile iterator's monotone repair (Sec. 4.4: crossing
quantiles replaced by their average, read as pool-adjacent-violators with
equal weights) and of the knot error the drivers report.

The iterator alone (pr_quantile_jump) is compared bit for bit with the
oracle on knot vectors built to cross after the add/subtract: isolated
crossings, long decreasing runs, hundreds of clusters, ties and near ties.
Whole parareal runs (plain and batched drivers) are compared with the
oracle's iteration on a small workload whose serial chain does cross: a
coarse grid of ten cells under 300 quantile levels, where the oracle itself
is checked to pool three or more knots in some link.  The error values of
the plain driver are compared with the oracle's RMS knot error of the same
states."""
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
    stream = torch.cuda.Stream()  # the batched driver's graph mode needs a non-default stream
    with torch.cuda.stream(stream):
        yield torch
    torch.cuda.synchronize()


def _longest_pool(v):
    """Longest run of the repaired vector made of one pool of distinct inputs."""
    out = OI.pava(np.asarray(v, dtype=np.float64).copy())
    best, cur = 1, 1
    for j in range(1, len(out)):
        if out[j] == out[j - 1] and v[j] != v[j - 1]:
            cur += 1
        else:
            best, cur = max(best, cur), 1
    return max(best, cur)


def _jump_cases():
    """(q_c_next, q_f, q_c_star) triples of rows of Q + 1 knots; the sum
    q_f + (q_c_next - q_c_star) crosses in the named ways."""
    rng = np.random.default_rng(29)
    cases = []
    Q = 100
    qf = np.sort(rng.uniform(-2.0, 2.0, Q + 1))
    qcs = np.sort(rng.uniform(-2.0, 2.0, Q + 1))
    cases.append(("monotone", qcs + 0.01, qf, qcs))
    d = np.zeros(Q + 1)
    d[[7, 40, 41, 77]] = [-0.3, 0.25, -0.5, -1.0]
    cases.append(("isolated", qcs + d, qf, qcs))
    d = np.zeros(Q + 1)
    d[30:80] = -np.linspace(0.0, 4.0, 50)           # one long decreasing run
    cases.append(("long run", qcs + d, qf, qcs))
    Q2 = 2047
    qf2 = np.sort(rng.uniform(-2.0, 2.0, Q2 + 1))
    qcs2 = np.sort(rng.uniform(-2.0, 2.0, Q2 + 1))
    d2 = np.zeros(Q2 + 1)
    d2[1::2] = -3e-3 * rng.random(Q2 // 2 + 1)[: len(d2[1::2])]   # a crossing every other knot: ~1000 clusters
    cases.append(("zig-zag", qcs2 + d2, qf2, qcs2))
    t = np.repeat(np.round(rng.uniform(-1, 1, 34), 1), 3)[: Q + 1]
    cases.append(("ties", np.zeros(Q + 1), np.sort(t)[::-1].copy(), np.zeros(Q + 1)))
    base = np.repeat(np.sort(np.round(rng.random(17), 2)), 6)[: Q + 1]
    near = base + rng.integers(-3, 4, base.size) * np.spacing(base)
    cases.append(("near ties", np.zeros(Q + 1), near, np.zeros(Q + 1)))
    thirds = (np.arange(Q + 1)[::-1] / 3.0).copy()
    cases.append(("thirds", thirds, np.zeros(Q + 1), np.zeros(Q + 1) + 0.1))
    return cases


@pytest.mark.parametrize("case", range(7))
def test_quantile_jump_bitwise(torch_dev, case):
    torch = torch_dev
    name, qcn, qf, qcs = _jump_cases()[case]
    L = len(qf)
    _say(f"quantile jump {name} L={L}")
    v = qf + (qcn - qcs)
    if name != "monotone":
        assert np.any(v[:-1] > v[1:]), name
    if name in ("long run", "zig-zag", "thirds"):
        assert _longest_pool(v) >= 3, name
    ref = OI.j_quantile(qcn, qf, qcs)
    rows = [torch.from_numpy(np.ascontiguousarray(np.stack([a, a]))).cuda() for a in (qcn, qf, qcs)]
    out = torch.empty((2, L), dtype=torch.float64, device="cuda")
    pr.pr_quantile_jump(rows[0], rows[1], rows[2], 2, L - 1, out)
    # in place over q_f, row for row
    pr.pr_quantile_jump(rows[0], rows[1], rows[2], 2, L - 1, rows[1])
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for r in range(2):
        assert np.array_equal(got[r], ref), (name, np.abs(got[r] - ref).max())
    assert np.array_equal(rows[1].cpu().numpy()[0], ref)
    assert np.all(np.diff(ref) >= 0.0)


def test_quantile_jump_iterator_property(torch_dev):
    """J(a, f, a) = f bit for bit for monotone f (eq. (iterator_property))."""
    torch = torch_dev
    rng = np.random.default_rng(31)
    k, Q = 5, 300
    f = np.sort(rng.normal(0.0, 1.0, (k, Q + 1)), axis=1)
    a = rng.normal(0.0, 3.0, (k, Q + 1))
    tf, ta = torch.from_numpy(f).cuda(), torch.from_numpy(a).cuda()
    out = torch.empty_like(tf)
    pr.pr_quantile_jump(ta, tf, ta, k, Q, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), f)


# ---------------------------------------------------------------------------
# whole runs whose serial chain crosses
# ---------------------------------------------------------------------------
CFG = dict(lam=1.0, beta=2.0, eps=0.1, n=500, dt=1e-3, T=0.6, K=6, cells=10, nq=300)


def _spy_oracle(sde, seed, inst, n, T, dt, K, cells, nq, reuse=False):
    """The oracle's iteration with every link's pre-repair vector recorded."""
    seen = []

    def jump(a, f, c):
        seen.append(np.asarray(f) + (np.asarray(a) - np.asarray(c)))
        return OI.j_quantile(a, f, c)

    po, hp = OI.micmac_parareal(sde, seed, inst, n, T, dt, K, OC.Grid(cells), nq, reuse_coarse=reuse)
    po.jump = jump
    return po, hp, seen


@pytest.mark.parametrize("reuse", [False, True])
def test_parareal_with_repair_matches_oracle(torch_dev, reuse):
    """Knots and states of every time point within 1e-10 / 1e-9 of the
    oracle after each of three iterations, on a workload whose chain pools
    three or more knots; the reported errors equal the oracle's RMS knot
    error of the GPU's states against the oracle's serial run (1e-12
    relative)."""
    torch = torch_dev
    c = CFG
    _say(f"parareal with repair reuse={reuse}")
    S = int(round(c["T"] / c["dt"]))
    sde = pr.Sde(lam=c["lam"], eps=c["eps"], beta=c["beta"])
    flags = pr.PR_REUSE_COARSE if reuse else 0
    h = pr.pr_parareal_create(sde, pr.Schedule(S, c["K"], c["T"] / S), pr.Grid(n_cells=c["cells"], n_q=c["nq"]),
                              0, 0, c["n"], flags)
    try:
        po, hp, seen = _spy_oracle(OP.Sde(lam=c["lam"], eps=c["eps"], beta=c["beta"]), 0, 0, c["n"], c["T"],
                                   c["dt"], c["K"], c["cells"], c["nq"], reuse)
        _, q_ref = OI.sequential_reference(hp, c["K"], c["nq"])
        qref = torch.from_numpy(np.ascontiguousarray(np.stack(q_ref))).cuda()
        for it in range(3):
            err = np.zeros(2)
            pr.pr_parareal_iterate(h, 1, q_ref=qref, err_out=err)
            po.iterate()
            qs = []
            for t in range(c["K"] + 1):
                x = torch.empty(c["n"], dtype=torch.float64, device="cuda")
                q = torch.empty(c["nq"] + 1, dtype=torch.float64, device="cuda")
                pr.pr_parareal_state(h, t, x=x, q=q)
                torch.cuda.synchronize()
                qg, xg = q.cpu().numpy(), x.cpu().numpy()
                qo = po.u[t].restricted(c["nq"])[0]
                assert np.abs(qg - qo).max() < 1e-10, (it, t, np.abs(qg - qo).max())
                assert np.abs(xg - po.u[t].x).max() < 1e-9, (it, t)
                qs.append(qg)
            e = [OI.quantile_error(qs[t], q_ref[t]) for t in range(c["K"] + 1)]
            assert e[-1] > 0.0 and max(e) > 0.0
            assert abs(err[0] - e[-1]) <= 1e-12 * e[-1], (it, err[0], e[-1])
            assert abs(err[1] - max(e)) <= 1e-12 * max(e), (it, err[1], max(e))
        assert max(_longest_pool(v) for v in seen) >= 3
        assert sum(1 for v in seen if np.any(v[:-1] > v[1:])) >= 5
    finally:
        pr.pr_parareal_destroy(h)


BATCH = [(0.05, 1.3, 600, 4, 0.2), (0.1, 0.7, 500, 6, 0.6), (0.02, 1.9, 800, 3, 0.3)]
BATCH_IDS = [11, 3, 40]


@pytest.mark.parametrize("mode", [pr.PR_LAUNCH_BATCHED, pr.PR_LAUNCH_GRAPH])
def test_batch_with_repair_matches_oracle(torch_dev, mode):
    """The batched driver's per-instance chains (one workgroup each) on
    instances whose chains pool knots: every instance's knots and states
    against the oracle after two iterations."""
    torch = torch_dev
    _say(f"batch with repair mode={mode}")
    cells, nq = 10, 300
    sdes, scheds, ns = [], [], []
    for eps, lam, n, K, T in BATCH:
        dt = eps / 20
        S = int(round(T / dt))
        sdes.append(pr.Sde(lam=lam, eps=eps, beta=2.0))
        scheds.append(pr.Schedule(S, K, T / S))
        ns.append(n)
    h = pr.pr_parareal_batch_create(sdes, scheds, ns, pr.Grid(n_cells=cells, n_q=nq), 7, instances=BATCH_IDS)
    try:
        pr.pr_parareal_batch_iterate(h, 2, mode)
        pools = []
        for i, ((eps, lam, n, K, T), iid) in enumerate(zip(BATCH, BATCH_IDS)):
            po, _, seen = _spy_oracle(OP.Sde(lam=lam, eps=eps, beta=2.0), 7, iid, n, T, eps / 20, K, cells, nq)
            po.iterate()
            po.iterate()
            pools.append(max(_longest_pool(v) for v in seen))
            for t in range(K + 1):
                x = torch.empty(n, dtype=torch.float64, device="cuda")
                q = torch.empty(nq + 1, dtype=torch.float64, device="cuda")
                pr.pr_parareal_batch_state(h, i, t, x=x, q=q)
                torch.cuda.synchronize()
                qo = po.u[t].restricted(nq)[0]
                assert np.abs(q.cpu().numpy() - qo).max() < 1e-10, (iid, t)
                assert np.abs(x.cpu().numpy() - po.u[t].x).max() < 1e-9, (iid, t)
        assert max(pools) >= 3
    finally:
        pr.pr_parareal_batch_destroy(h)
