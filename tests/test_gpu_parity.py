"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Bit-exact for orders, ranks, histograms and the
formulas evaluated in the same order; FP64 within 1e-10 for knots and
moments (the tolerance of the method's parity target); per-particle
trajectories within 1e-12 after a slice (normals differ by the last bits of
the device and host log/sin/cos)."""
import sys

import numpy as np
import pytest

import paper_1912_09240_amd as pr
from oracle import coarse as OC
from oracle import iterate as OI
from oracle import particles as OP
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


def _sync(torch):
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# noise, initial ensemble, fine propagator
# ---------------------------------------------------------------------------
def test_coupling_bitwise(torch_dev):
    torch = torch_dev
    _say("coupling d=32")
    a = torch.zeros(32, dtype=torch.float64, device="cuda")
    pr.pr_draw_coupling(0, 0, 32, a)
    _sync(torch)
    assert np.array_equal(a.cpu().numpy(), OP.coupling(0, 0, 32))


@pytest.mark.parametrize("d,n", [(1, 10_007), (3, 1_000), (32, 513)])
def test_init_ensemble(torch_dev, d, n):
    torch = torch_dev
    _say(f"init d={d} n={n}")
    a_np = OP.coupling(7, 3, d) if d > 1 else None
    a = torch.from_numpy(a_np).cuda() if a_np is not None else None
    s = pr.Sde(beta=2.0, d=d, a=a)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    y = torch.empty((d, n), dtype=torch.float64, device="cuda")
    pr.pr_init_ensemble(s, 7, 3, n, x, y)
    _sync(torch)
    xo, yo = OP.init_ensemble(OP.Sde(beta=2.0, d=d, a=a_np), 7, 3, n)
    xg, yg = x.cpu().numpy(), y.cpu().numpy()
    if d == 1:
        # x = z0 / 2, y = x + z1 / sqrt(2): the normals themselves, to the
        # oracle's rounding of the angle (~1e-15 of the radius r)
        r = np.hypot(2 * xo, (yo[0] - xo) * np.sqrt(2.0))
        assert np.all(np.abs(xg - xo) <= 0.5e-15 * (1 + r))
        assert np.all(np.abs(yg[0] - yo[0]) <= 2e-15 * (1 + r))
    assert np.abs(xg - xo).max() < 1e-14
    assert np.abs(yg - yo).max() < 1e-14


@pytest.mark.parametrize("d,n,S,K,dt,eps", [(1, 4_099, 300, 3, 1e-3, 0.1), (1, 10_000, 1000, 10, 1e-3, 0.1),
                                             (32, 700, 120, 2, 1e-4, 0.01), (2, 257, 50, 5, 1e-3, 0.05)])
def test_fine_propagate_all_slices(torch_dev, d, n, S, K, dt, eps):
    """All K slices in one launch, each from its own start state, against the
    oracle slice by slice."""
    torch = torch_dev
    _say(f"fine d={d} n={n} S={S} K={K}")
    a_np = OP.coupling(0, 0, d) if d > 1 else None
    so = OP.Sde(lam=1.0, eps=eps, beta=2.0, d=d, a=a_np)
    x0, y0 = OP.init_ensemble(so, 0, 0, n)
    # distinct start states per slice: the ensemble shifted by the slice index
    xs = np.stack([x0 + 0.1 * k for k in range(K)])
    ys = np.stack([y0 - 0.05 * k for k in range(K)])
    x = torch.from_numpy(xs.copy()).cuda()
    y = torch.from_numpy(ys.copy()).cuda()
    a = torch.from_numpy(a_np).cuda() if a_np is not None else None
    pr.pr_fine_propagate(pr.Sde(lam=1.0, eps=eps, beta=2.0, d=d, a=a), pr.Schedule(S, K, dt), 0, 0, n, 0, K, x, y)
    _sync(torch)
    xg, yg = x.cpu().numpy(), y.cpu().numpy()
    b = OI.slice_bounds(S, K)
    for k in range(K):
        xr, yr = OP.em_propagate(so, 0, 0, xs[k], ys[k], b[k], b[k + 1], dt)
        assert np.abs(xg[k] - xr).max() < 1e-12 * max(1.0, np.abs(xr).max()), k
        assert np.abs(yg[k] - yr).max() < 1e-12 * max(1.0, np.abs(yr).max()), k


def test_fine_large_workload_sampled(torch_dev):
    """The large workload's launch (P = 2^20, all 64 slices of 1e5 steps of
    dt = 1e-4 in one launch, 2 particles per thread), each slice from its own
    start state, against the oracle on 32 particles of every slice (the last
    32 of the last slice included)."""
    torch = torch_dev
    cfg = inputs.CFG_LARGE
    n, K = cfg["n"], cfg["K"]
    S = int(round(cfg["T"] / cfg["dt"]))
    dt = cfg["T"] / S
    _say(f"fine large n={n} K={K} S={S}")
    so = OP.Sde(lam=cfg["lam"], eps=cfg["eps"], beta=cfg["beta"])
    x0, y0 = OP.init_ensemble(so, 0, 0, n)
    x = torch.from_numpy(np.stack([x0 + 0.01 * k for k in range(K)])).cuda()
    y = torch.from_numpy(np.stack([y0[0] - 0.01 * k for k in range(K)])).cuda()
    pr.pr_fine_propagate(pr.Sde(lam=cfg["lam"], eps=cfg["eps"], beta=cfg["beta"]), pr.Schedule(S, K, dt), 0, 0, n,
                         0, K, x, y)
    _sync(torch)
    b = OI.slice_bounds(S, K)
    for k in range(K):
        p0 = n - 32 if k == K - 1 else (k * 16_381) % (n - 32)
        xg = x[k, p0:p0 + 32].cpu().numpy()
        yg = y[k, p0:p0 + 32].cpu().numpy()
        xr, yr = OP.em_propagate(so, 0, 0, x0[p0:p0 + 32] + 0.01 * k, y0[:, p0:p0 + 32] - 0.01 * k, b[k], b[k + 1],
                                 dt, p0=p0)
        assert np.abs(xg - xr).max() < 1e-12 * max(1.0, np.abs(xr).max()), k
        assert np.abs(yg - yr[0]).max() < 1e-12 * max(1.0, np.abs(yr).max()), k


def test_fine_high_dim_workload_sampled(torch_dev):
    """The fast part in R^32 at its full size and launch (P = 2^20, all 32
    slices of 5e4 steps of dt = 1e-4 in one launch, FP64), each slice from
    its own start state, against the oracle on 8 particles of every slice
    (the last 8 of the last slice included)."""
    torch = torch_dev
    n, K, d, S, dt, eps = 2 ** 20, 32, 32, 50_000, 1e-4, 0.01
    _say(f"fine d=32 full size n={n} K={K} S={S}")
    a_np = OP.coupling(0, 0, d)
    so = OP.Sde(lam=1.0, eps=eps, beta=2.0, d=d, a=a_np)
    a = torch.from_numpy(a_np).cuda()
    sde = pr.Sde(lam=1.0, eps=eps, beta=2.0, d=d, a=a)
    x0 = torch.empty(n, dtype=torch.float64, device="cuda")
    y0 = torch.empty((d, n), dtype=torch.float64, device="cuda")
    pr.pr_init_ensemble(sde, 0, 0, n, x0, y0)
    shift = 0.01 * torch.arange(K, dtype=torch.float64, device="cuda")
    x = (x0.unsqueeze(0) + shift[:, None]).contiguous()
    y = (y0.unsqueeze(0) - shift[:, None, None]).contiguous()
    pr.pr_fine_propagate(sde, pr.Schedule(S, K, dt), 0, 0, n, 0, K, x, y)
    _sync(torch)
    x0h, y0h = OP.init_ensemble(so, 0, 0, n)
    assert np.abs(x0.cpu().numpy() - x0h).max() < 1e-14
    b = OI.slice_bounds(S, K)
    for k in range(K):
        p0 = n - 8 if k == K - 1 else (k * 32_749) % (n - 8)
        xg = x[k, p0:p0 + 8].cpu().numpy()
        yg = y[k, :, p0:p0 + 8].cpu().numpy()
        xr, yr = OP.em_propagate(so, 0, 0, x0h[p0:p0 + 8] + 0.01 * k, y0h[:, p0:p0 + 8] - 0.01 * k, b[k], b[k + 1],
                                 dt, p0=p0)
        assert np.abs(xg - xr).max() < 1e-12 * max(1.0, np.abs(xr).max()), k
        assert np.abs(yg - yr).max() < 1e-12 * max(1.0, np.abs(yr).max()), k


def test_fine_subrange_and_in_place(torch_dev):
    """Slices [2, 4) of a 5-slice schedule on their own give the same numbers
    as inside a full launch (counter-based noise keyed by the global step)."""
    torch = torch_dev
    _say("fine subrange")
    n, S, K, dt = 3000, 500, 5, 1e-3
    so = OP.Sde()
    x0, y0 = OP.init_ensemble(so, 1, 0, n)
    xs = np.stack([x0] * K)
    ys = np.stack([y0] * K)
    xa, ya = torch.from_numpy(xs.copy()).cuda(), torch.from_numpy(ys.copy()).cuda()
    pr.pr_fine_propagate(pr.Sde(), pr.Schedule(S, K, dt), 1, 0, n, 0, K, xa, ya)
    xb, yb = torch.from_numpy(xs[2:4].copy()).cuda(), torch.from_numpy(ys[2:4].copy()).cuda()
    pr.pr_fine_propagate(pr.Sde(), pr.Schedule(S, K, dt), 1, 0, n, 2, 2, xb, yb)
    _sync(torch)
    assert torch.equal(xa[2:4], xb) and torch.equal(ya[2:4], yb)


def test_fine_fp32_error_vs_fp64_oracle(torch_dev):
    """FP32 stepping: its normals come from 24-bit uniforms, so it is a
    different discretisation of the same law; report and bound its knot error
    against the FP64 oracle (statistical, not per-particle)."""
    torch = torch_dev
    _say("fine fp32")
    n, S, dt = 200_000, 200, 1e-3
    so = OP.Sde()
    x0, y0 = OP.init_ensemble(so, 2, 0, n)
    x = torch.from_numpy(x0.astype(np.float32)).cuda()
    y = torch.from_numpy(y0.astype(np.float32)).cuda()
    pr.pr_fine_propagate(pr.Sde(precision=pr.PR_F32), pr.Schedule(S, 1, dt), 2, 0, n, 0, 1, x, y)
    _sync(torch)
    xr, _ = OP.em_propagate(so, 2, 0, x0, y0, 0, S, dt)
    q32 = OR.hazen_knots(np.sort(x.cpu().numpy().astype(np.float64)), 100)
    q64 = OR.hazen_knots(np.sort(xr), 100)
    err = np.abs(q32 - q64)[1:-1].max()
    _say(f"fp32 stepping: max interior knot error vs FP64 oracle = {err:.3e}")
    assert err < 0.02


@pytest.mark.parametrize("d,n,S,K,dt,eps", [(1, 4_099, 300, 3, 1e-3, 0.1), (32, 700, 120, 2, 1e-4, 0.01),
                                             (2, 257, 50, 5, 1e-3, 0.05)])
def test_fine_fp32_per_particle(torch_dev, d, n, S, K, dt, eps):
    """FP32 stepping particle by particle against the oracle run with the
    same normals (the 24- and 28-bit uniforms of the same words) in double
    precision.  They differ only by float rounding: per step at most six
    roundings of the state (6 * 2^-24 per unit of |state|) and the float
    transform's error (a few 2^-24 of |z| <= 5.9, times sqrt(2 dt/beta) or
    sqrt(2 dt/(beta eps)) <= 0.1), under 5e-7 per unit, grown by at most
    e^{2T} < 1.9 along a slice of T <= 0.3; so 1e-6 per step and unit.  The
    rounding of u = (k + 1/2) 2^-24 to a float moves the radius by up to
    2^-12 / sqrt(2) for the rare u within a few 2^-24 of 1: 2e-5 more after
    the factor 0.1.  A wrong bit, word, coefficient or sign moves a particle
    by ~sqrt(2 dt/beta) = 0.03 (or 0.01 for dt = 1e-4) in one step."""
    torch = torch_dev
    _say(f"fine fp32 d={d} n={n} S={S} K={K}")
    a_np = OP.coupling(0, 0, d) if d > 1 else None
    so = OP.Sde(lam=1.0, eps=eps, beta=2.0, d=d, a=a_np)
    x0, y0 = OP.init_ensemble(so, 0, 0, n)
    xs = np.stack([x0 + 0.1 * k for k in range(K)]).astype(np.float32)
    ys = np.stack([y0 - 0.05 * k for k in range(K)]).astype(np.float32)
    x = torch.from_numpy(xs.copy()).cuda()
    y = torch.from_numpy(ys.copy()).cuda()
    a = torch.from_numpy(a_np).cuda() if a_np is not None else None
    sde = pr.Sde(lam=1.0, eps=eps, beta=2.0, d=d, a=a, precision=pr.PR_F32)
    pr.pr_fine_propagate(sde, pr.Schedule(S, K, dt), 0, 0, n, 0, K, x, y)
    _sync(torch)
    xg, yg = x.cpu().numpy().astype(np.float64), y.cpu().numpy().astype(np.float64)
    b = OI.slice_bounds(S, K)
    worst = 0.0
    for k in range(K):
        xr, yr = OP.em_propagate(so, 0, 0, xs[k].astype(np.float64), ys[k].astype(np.float64), b[k], b[k + 1], dt,
                                 f32_noise=True)
        steps = b[k + 1] - b[k]
        scale = max(1.0, np.abs(xr).max(), np.abs(yr).max())
        tol = 1e-6 * steps * scale + 2e-5
        ex, ey = np.abs(xg[k] - xr).max(), np.abs(yg[k] - yr).max()
        worst = max(worst, ex / tol, ey / tol)
        assert ex < tol and ey < tol, (k, ex, ey, tol)
        # the typical particle is much closer: rounding errors of both signs
        assert np.sqrt(np.mean((xg[k] - xr) ** 2)) < 1e-6 * np.sqrt(steps) * scale, k
    _say(f"fp32 per particle: worst error / tolerance = {worst:.3e}")


# ---------------------------------------------------------------------------
# restriction
# ---------------------------------------------------------------------------
def _restrict_gpu(torch, xs_np, nq, precision=pr.PR_F64, hist_grid=None):
    k, n = xs_np.shape
    x = torch.from_numpy(xs_np).cuda()
    ws = torch.empty(pr.pr_restrict_workspace_size(n, k, precision), dtype=torch.uint8, device="cuda")
    q = torch.empty((k, nq + 1), dtype=torch.float64, device="cuda")
    rank = torch.empty((k, n), dtype=torch.int32, device="cuda")
    perm = torch.empty((k, n), dtype=torch.int32, device="cuda")
    xsorted = torch.empty((k, n), dtype=torch.float64, device="cuda")
    mom = torch.empty((k, 4), dtype=torch.float64, device="cuda")
    hist = torch.empty((k, hist_grid.n_cells), dtype=torch.int32, device="cuda") if hist_grid else None
    pr.pr_restrict_quantiles(x, precision, n, k, nq, q, ws, rank=rank, perm=perm, x_sorted=xsorted, moments=mom,
                             hist=hist, hist_grid=hist_grid)
    torch.cuda.synchronize()
    out = dict(q=q.cpu().numpy(), rank=rank.cpu().numpy().view(np.uint32), perm=perm.cpu().numpy().view(np.uint32),
               xs=xsorted.cpu().numpy(), mom=mom.cpu().numpy())
    if hist is not None:
        out["hist"] = hist.cpu().numpy().view(np.uint32)
    return out


@pytest.mark.parametrize("k,n", [(1, 1), (2, 2), (3, 17), (2, 4096), (2, 4097), (5, 10_007), (3, 70_001)])
def test_restrict_identical_inputs(torch_dev, k, n):
    torch = torch_dev
    _say(f"restrict k={k} n={n}")
    xs = inputs.slow_values(10 + n, k, n)
    g = pr.Grid(n_cells=200)
    out = _restrict_gpu(torch, xs, 100, hist_grid=g)
    for s in range(k):
        perm, rank, srt = OR.sort_ranks(xs[s])
        assert np.array_equal(out["perm"][s], perm), s
        assert np.array_equal(out["rank"][s], rank), s
        assert np.array_equal(out["xs"][s].view(np.uint64), srt.view(np.uint64)), s
        assert np.array_equal(out["q"][s], OR.hazen_knots(srt, 100)), s
        mo = OR.moments(xs[s])
        assert np.all(np.abs(out["mom"][s] - mo) <= 1e-12 * np.maximum(1.0, np.abs(mo))), s
        assert np.array_equal(out["hist"][s], OR.histogram(xs[s], 200, -3.0, 3.0)), s


@pytest.mark.parametrize("k,n", [(5000, 3), (700, 65)])
def test_restrict_many_small_segments(torch_dev, k, n):
    """Thousands of ensembles of a few particles each (one partial tile per
    segment, runs of equal high halves across the whole segment)."""
    torch = torch_dev
    _say(f"restrict many segments k={k} n={n}")
    xs = inputs.slow_values(40 + k, k, n, ties=False)
    xs[: k // 2, : min(n, 3)] = 0.25  # exact ties inside a segment
    out = _restrict_gpu(torch, xs, 10)
    for s in range(0, k, max(1, k // 97)):
        perm, rank, srt = OR.sort_ranks(xs[s])
        assert np.array_equal(out["perm"][s], perm), s
        assert np.array_equal(out["rank"][s], rank), s
        assert np.array_equal(out["xs"][s].view(np.uint64), srt.view(np.uint64)), s
        assert np.array_equal(out["q"][s], OR.hazen_knots(srt, 10)), s


@pytest.mark.parametrize("k,n,ties,prec", [(1, 1, False, pr.PR_F64), (3, 4097, False, pr.PR_F64),
                                           (4, 70_001, True, pr.PR_F64), (2, 2 ** 20, False, pr.PR_F64),
                                           (2, 2 ** 20, True, pr.PR_F64), (1, 2 ** 20 + 1, False, pr.PR_F64),
                                           (1, 2 ** 20 + 2 ** 17, False, pr.PR_F64),
                                           (2, 2 ** 16, False, pr.PR_F64), (2, 2 ** 16 - 1, False, pr.PR_F64),
                                           (3, 4097, True, pr.PR_F32), (2, 2 ** 20, False, pr.PR_F32),
                                           (1, 2 ** 20 + 1, True, pr.PR_F32)])
def test_restrict_rank_only(torch_dev, k, n, ties, prec):
    """Ranks asked for alone, as the parareal drivers do: up to 2^20 keys per
    segment they go through the staging buffer, beyond by direct stores; for
    FP64 keys the runs of hundreds of signed zeros of ties=True hand the
    ranks to the complete sort, and ensembles above 2^20 + 2^16 keys are
    sorted by the radix passes from the start, as are those below 2^16 (the
    two sizes at that edge: 2^16 by splitters in 16 buckets, 2^16 - 1 by
    radix passes)."""
    torch = torch_dev
    _say(f"restrict rank only k={k} n={n} ties={ties} precision={prec}")
    xs = inputs.slow_values(300 + n % 1000, k, n, ties=ties)
    if prec == pr.PR_F32:
        xs = xs.astype(np.float32)
    x = torch.from_numpy(xs).cuda()
    ws = torch.empty(pr.pr_restrict_workspace_size(n, k, prec), dtype=torch.uint8, device="cuda")
    q = torch.empty((k, 11), dtype=torch.float64, device="cuda")
    rank = torch.empty((k, n), dtype=torch.int32, device="cuda")
    pr.pr_restrict_quantiles(x, prec, n, k, 10, q, ws, rank=rank)
    torch.cuda.synchronize()
    rk, qg = rank.cpu().numpy().view(np.uint32), q.cpu().numpy()
    for s in range(k):
        _, ref, srt = OR.sort_ranks(xs[s].astype(np.float64))
        assert np.array_equal(rk[s], ref), s
        assert np.array_equal(qg[s], OR.hazen_knots(srt, 10)), s


def test_restrict_large_segments(torch_dev):
    torch = torch_dev
    n, k = 2 ** 20, 3
    _say(f"restrict large k={k} n={n}")
    xs = inputs.slow_values(99, k, n)
    out = _restrict_gpu(torch, xs, 100)
    for s in range(k):
        perm, rank, srt = OR.sort_ranks(xs[s])
        assert np.array_equal(out["perm"][s], perm)
        assert np.array_equal(out["rank"][s], rank)
        assert np.array_equal(out["q"][s], OR.hazen_knots(srt, 100))


def _splitter_case(case, k, n):
    rng = np.random.default_rng(700 + case)
    x = rng.normal(0.0, 1.0, (k, n))
    if case == 1:    # every key equal: one bucket holds the whole ensemble
        x[:] = 0.625
    elif case == 2:  # one far outlier stretches the last bucket's value range
        x[:, 17] = 1e300
    elif case == 3:  # runs of 300 equal values inside buckets
        x = np.round(rng.normal(0.0, 1.0, (k, n)) * 60.0) / 60.0
    elif case == 4:  # infinities and signed zeros among smooth values
        x[:, ::997] = np.inf
        x[:, 5::991] = -np.inf
        x[:, 7::89] = -0.0
        x[:, 11::97] = 0.0
    elif case == 5:  # a few copies of most values, spread over every bucket
        x = np.round(rng.normal(0.0, 1.0, (k, n)) * 8000.0) / 8000.0
    return np.ascontiguousarray(x)


@pytest.mark.parametrize("case", range(6))
def test_restrict_splitter_cases(torch_dev, case):
    """Ensembles of 2^17 particles (sorted by splitters and buckets where
    every bucket fits, by the complete radix sort otherwise): smooth values,
    all equal, a far outlier, long runs of ties, infinities and signed zeros,
    a few copies of most values.
    Every output bit for bit against the oracle's stable sort."""
    torch = torch_dev
    k, n = 2, 2 ** 17
    _say(f"restrict splitter case {case}")
    xs = _splitter_case(case, k, n)
    out = _restrict_gpu(torch, xs, 100)
    for s in range(k):
        perm, rank, srt = OR.sort_ranks(xs[s])
        assert np.array_equal(out["perm"][s], perm), s
        assert np.array_equal(out["rank"][s], rank), s
        assert np.array_equal(out["xs"][s].view(np.uint64), srt.view(np.uint64)), s
        assert np.array_equal(out["q"][s], OR.hazen_knots(srt, 100)), s


def test_restrict_fp32(torch_dev):
    torch = torch_dev
    _say("restrict fp32")
    xs = inputs.slow_values(5, 3, 9_001).astype(np.float32)
    out = _restrict_gpu(torch, xs, 64, precision=pr.PR_F32)
    for s in range(3):
        perm, rank, srt = OR.sort_ranks(xs[s].astype(np.float64))
        assert np.array_equal(out["perm"][s], perm)
        assert np.array_equal(out["rank"][s], rank)
        assert np.array_equal(out["q"][s], OR.hazen_knots(srt, 64))
        mo = OR.moments(xs[s].astype(np.float64))
        assert np.all(np.abs(out["mom"][s] - mo) <= 1e-12 * np.maximum(1.0, np.abs(mo)))


# ---------------------------------------------------------------------------
# matching
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k,n,nq", [(1, 1, 2), (3, 1_001, 100), (4, 65_537, 100), (2, 5_000, 7)])
def test_match_identical_inputs(torch_dev, k, n, nq):
    torch = torch_dev
    _say(f"match k={k} n={n}")
    xs = inputs.slow_values(3 + n, k, n, ties=False)
    rk = inputs.ranks(4 + n, k, n)
    qt = inputs.monotone_knots(5, k, nq)
    qp = inputs.monotone_knots(6, k, nq)
    x = torch.from_numpy(xs).cuda()
    out = torch.empty_like(x)
    pr.pr_match_quantiles(torch.from_numpy(qt).cuda(), torch.from_numpy(qp).cuda(),
                          torch.from_numpy(rk.view(np.int32)).cuda(), n, k, nq, x, out)
    same = torch.empty_like(x)
    qpd = torch.from_numpy(qp).cuda()
    pr.pr_match_quantiles(qpd, qpd, torch.from_numpy(rk.view(np.int32)).cuda(), n, k, nq, x, same)
    torch.cuda.synchronize()
    og = out.cpu().numpy()
    for s in range(k):
        ref = OI.match_quantiles(xs[s], rk[s], qt[s], qp[s])
        assert np.array_equal(og[s], ref), s
    assert torch.equal(same, x)  # projection, bitwise


# ---------------------------------------------------------------------------
# coarse propagator
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("I,S,K,dt", [(200, 1000, 10, 1e-3), (1024, 100_000, 64, 1e-4)])
def test_coarse_matches_oracle(torch_dev, I, S, K, dt):
    torch = torch_dev
    _say(f"coarse I={I}")
    sde = pr.Sde()
    h = pr.pr_coarse_create(sde, pr.Schedule(S, K, dt), pr.Grid(n_cells=I))
    try:
        og = OC.Grid(I)
        prop = OC.Propagator(og, OP.Sde())
        b = OI.slice_bounds(S, K)
        for s in (0, K - 1):
            Ep = pr.pr_coarse_matrix(h, s)
            torch.cuda.synchronize()
            Eg = _copy_device(torch, Ep, I * I).reshape(I, I)
            Eo = prop.expm((b[s + 1] - b[s]) * dt)
            assert np.abs(Eg - Eo).max() < 1e-11, s
            assert np.abs(Eg.sum(0) - 1).max() < 1e-11, s
        qin = inputs.monotone_knots(8, K, 100, -2.0, 2.0)
        qg = torch.empty((K, 101), dtype=torch.float64, device="cuda")
        rho = torch.empty((K, I), dtype=torch.float64, device="cuda")
        pr.pr_coarse_fp_step(h, 0, K, torch.from_numpy(qin).cuda(), qg, rho)
        torch.cuda.synchronize()
        for s in range(K):
            E = prop.expm((b[s + 1] - b[s]) * dt)
            qo, ro = OC.coarse_step(qin[s], E, og)
            assert np.abs(rho.cpu().numpy()[s] - ro).max() < 1e-12, s
            assert np.abs(qg.cpu().numpy()[s] - qo).max() < 1e-10, s
    finally:
        pr.pr_coarse_destroy(h)


def _copy_device(torch, ptr, count):
    """Copy `count` doubles from a raw device pointer into numpy."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    out = np.empty(count, dtype=np.float64)
    rc = hip.hipMemcpy(ctypes.c_void_p(out.ctypes.data), ctypes.c_void_p(ptr), ctypes.c_size_t(count * 8),
                       ctypes.c_int(2))
    assert rc == 0
    return out


# ---------------------------------------------------------------------------
# parareal
# ---------------------------------------------------------------------------
def _gpu_parareal(torch, cfg, flags=0, seed=0):
    S = int(round(cfg["T"] / cfg["dt"]))
    sched = pr.Schedule(S, cfg["K"], cfg["T"] / S)
    grid = pr.Grid(n_cells=cfg["cells"], n_q=cfg["nq"])
    sde = pr.Sde(lam=cfg["lam"], eps=cfg["eps"], beta=cfg["beta"])
    h = pr.pr_parareal_create(sde, sched, grid, seed, 0, cfg["n"], flags)
    return h, sde, sched


def _gpu_states(torch, h, K, n, nq):
    xs, qs = [], []
    for t in range(K + 1):
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        q = torch.empty(nq + 1, dtype=torch.float64, device="cuda")
        pr.pr_parareal_state(h, t, x=x, q=q)
        xs.append(x)
        qs.append(q)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in xs], [q.cpu().numpy() for q in qs]


@pytest.mark.parametrize("reuse", [False, True])
def test_parareal_small_workload_matches_oracle(torch_dev, reuse):
    """The small workload (N = 1e4 particles, 10 slices, 200 cells, 100
    levels, 2 iterations) against the oracle's iteration: knots of every
    state within 1e-10 after the zeroth and each later iteration."""
    torch = torch_dev
    cfg = inputs.CFG_SMALL
    _say(f"parareal small reuse={reuse}")
    flags = pr.PR_REUSE_COARSE if reuse else 0
    h, _, _ = _gpu_parareal(torch, cfg, flags)
    try:
        po, hp = OI.micmac_parareal(OP.Sde(lam=cfg["lam"], eps=cfg["eps"], beta=cfg["beta"]), 0, 0, cfg["n"],
                                    cfg["T"], cfg["dt"], cfg["K"], OC.Grid(cfg["cells"]), cfg["nq"],
                                    reuse_coarse=reuse)
        for it in range(cfg["iters"] + 1):
            if it > 0:
                pr.pr_parareal_iterate(h, 1)
                po.iterate()
            xg, qg = _gpu_states(torch, h, cfg["K"], cfg["n"], cfg["nq"])
            for t in range(cfg["K"] + 1):
                qo = po.u[t].restricted(cfg["nq"])[0]
                err = np.abs(qg[t] - qo).max()
                assert err < 1e-10, (it, t, err)
                assert np.abs(xg[t] - po.u[t].x).max() < 1e-9, (it, t)
    finally:
        pr.pr_parareal_destroy(h)


@pytest.mark.parametrize("flags", [0, pr.PR_REUSE_COARSE, pr.PR_SKIP_CONVERGED])
def test_parareal_exactness_bitwise(torch_dev, flags):
    """After k iterations the states at t <= k equal the GPU's own serial
    fine run bitwise; after K iterations all do, and the knot error to the
    serial run is exactly 0."""
    torch = torch_dev
    cfg = dict(inputs.CFG_SMALL, n=3000, K=6, T=0.3)
    _say(f"parareal exactness flags={flags}")
    h, sde, sched = _gpu_parareal(torch, cfg, flags)
    n, K, nq = cfg["n"], cfg["K"], cfg["nq"]
    try:
        # serial reference on the GPU
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        pr.pr_init_ensemble(sde, 0, 0, n, x, y)
        ref = [x.clone()]
        qref = torch.empty((K + 1, nq + 1), dtype=torch.float64, device="cuda")
        ws = torch.empty(pr.pr_restrict_workspace_size(n, 1), dtype=torch.uint8, device="cuda")
        pr.pr_restrict_quantiles(x, pr.PR_F64, n, 1, nq, qref[0], ws)
        for s in range(K):
            pr.pr_fine_propagate(sde, sched, 0, 0, n, s, 1, x, y)
            ref.append(x.clone())
            pr.pr_restrict_quantiles(x, pr.PR_F64, n, 1, nq, qref[s + 1], ws)
        torch.cuda.synchronize()
        errs = np.zeros(2 * K)
        for k in range(1, K + 1):
            pr.pr_parareal_iterate(h, 1, q_ref=qref, err_out=errs[2 * (k - 1):])
            xg, _ = _gpu_states(torch, h, K, n, nq)
            for t in range(k + 1):
                assert np.array_equal(xg[t], ref[t].cpu().numpy()), (k, t)
        assert errs[-1] == 0.0 and errs[-2] == 0.0
        assert pr.pr_parareal_iteration(h) == K
    finally:
        pr.pr_parareal_destroy(h)


def test_parareal_large_workload_iteration(torch_dev):
    """The large workload as the benchmark runs it (P = 2^20, 64 slices of
    1e5 steps, 1024 cells, 100 levels): after one iteration the state at t_1
    is the fine propagation of X0 bitwise and its knots are the serial run's
    exactly (Sec. 3.3.3); every state's knots are non-decreasing,
    start and end at the state's extremes and agree with the Hazen knots the
    oracle takes of the same state."""
    torch = torch_dev
    cfg = inputs.CFG_LARGE
    n, K, nq = cfg["n"], cfg["K"], cfg["nq"]
    _say(f"parareal large n={n} K={K}")
    h, sde, sched = _gpu_parareal(torch, cfg)
    try:
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        pr.pr_init_ensemble(sde, 0, 0, n, x, y)
        qref = torch.zeros((K + 1, nq + 1), dtype=torch.float64, device="cuda")
        ws = torch.empty(pr.pr_restrict_workspace_size(n, 1), dtype=torch.uint8, device="cuda")
        pr.pr_restrict_quantiles(x, pr.PR_F64, n, 1, nq, qref[0], ws)
        pr.pr_fine_propagate(sde, sched, 0, 0, n, 0, 1, x, y)
        pr.pr_restrict_quantiles(x, pr.PR_F64, n, 1, nq, qref[1], ws)
        errs = np.zeros(2)
        pr.pr_parareal_iterate(h, 1, q_ref=qref, err_out=errs)
        xs = torch.empty(n, dtype=torch.float64, device="cuda")
        q = torch.empty(nq + 1, dtype=torch.float64, device="cuda")
        pr.pr_parareal_state(h, 1, x=xs, q=q)
        assert torch.equal(xs, x)
        assert torch.equal(q, qref[1])
        for t in (2, K // 2, K):
            pr.pr_parareal_state(h, t, x=xs, q=q)
            xn, qn = xs.cpu().numpy(), q.cpu().numpy()
            assert np.all(np.diff(qn) >= 0.0), t
            assert qn[0] == xn.min() and qn[-1] == xn.max(), t
            assert np.array_equal(qn, OR.hazen_knots(np.sort(xn), nq)), t
    finally:
        pr.pr_parareal_destroy(h)
