"""Profiling driver: runs one kernel group of the large workload once, so
that rocprofv3 counter passes cover a handful of dispatches.

    python -m paper_1912_09240_amd.profile_workload fine      # all 64 slices, one launch
    python -m paper_1912_09240_amd.profile_workload restrict  # sort of 64 x 2^20 keys with ranks
    python -m paper_1912_09240_amd.profile_workload match     # matching of 64 x 2^20 particles and the
                                                              # knots of the matched states
    python -m paper_1912_09240_amd.profile_workload copy      # device-to-device copy of 1 GiB
    python -m paper_1912_09240_amd.profile_workload hist      # histograms, marginal matching and
                                                              # stratified resampling, 64 x 2^20
    python -m paper_1912_09240_amd.profile_workload chem      # chemical-reaction fine launch (Table 1)
    python -m paper_1912_09240_amd.profile_workload adjoint   # differentiated form: forward with
                                                              # checkpoints, observables, reverse sweep
    python -m paper_1912_09240_amd.profile_workload batch     # batched form: creation (zeroth iteration)
                                                              # of 256 instances and one batched iteration

Large workload: lambda = 1, beta = 2, eps = 0.01, P = 2^20, dt = 1e-4, T = 10
(1e5 steps) in 64 slices, 100 quantile levels; the slice states start from
the initial ensemble.  Every group is preceded by one untimed run of itself.
"""
import sys

import torch

import paper_1912_09240_amd as pr

N, K, S, DT, NQ = 2 ** 20, 64, 100_000, 1e-4, 100


def _ensemble():
    sde = pr.Sde(lam=1.0, eps=0.01, beta=2.0)
    x0 = torch.empty(N, dtype=torch.float64, device="cuda")
    y0 = torch.empty(N, dtype=torch.float64, device="cuda")
    pr.pr_init_ensemble(sde, 0, 0, N, x0, y0)
    return sde, x0.repeat(K, 1).contiguous(), y0.repeat(K, 1).contiguous()


def fine():
    sde, x, y = _ensemble()
    sched = pr.Schedule(S, K, DT)
    for _ in range(2):
        xs, ys = x.clone(), y.clone()
        pr.pr_fine_propagate(sde, sched, 0, 0, N, 0, K, xs, ys)
        torch.cuda.synchronize()


def restrict():
    _, x, _ = _ensemble()
    ws = torch.empty(pr.pr_restrict_workspace_size(N, K), dtype=torch.uint8, device="cuda")
    q = torch.empty((K, NQ + 1), dtype=torch.float64, device="cuda")
    rank = torch.empty((K, N), dtype=torch.int32, device="cuda")
    for _ in range(2):
        pr.pr_restrict_quantiles(x, pr.PR_F64, N, K, NQ, q, ws, rank=rank)
        torch.cuda.synchronize()


def match():
    _, x, _ = _ensemble()
    ws = torch.empty(pr.pr_restrict_workspace_size(N, K), dtype=torch.uint8, device="cuda")
    q = torch.empty((K, NQ + 1), dtype=torch.float64, device="cuda")
    rank = torch.empty((K, N), dtype=torch.int32, device="cuda")
    pr.pr_restrict_quantiles(x, pr.PR_F64, N, K, NQ, q, ws, rank=rank)
    qt = q + 0.01
    qm = torch.empty_like(q)
    flag = torch.zeros((1,), dtype=torch.int32, device="cuda")
    for _ in range(2):
        pr.pr_match_quantiles(qt, q, rank, N, K, NQ, x, x)
        pr.pr_match_knots(qt, q, N, K, NQ, ws, qm, flag)
        torch.cuda.synchronize()


def copy():
    a = torch.empty(2 ** 27, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
        torch.cuda.synchronize()


def hist():
    """Histogram restriction of the 64 ensembles (1024 cells on [-3, 3]),
    then the fast-marginal matching and the stratified resampling of every
    ensemble against its histogram shifted by five cells."""
    _, x, y = _ensemble()
    grid = pr.Grid(n_cells=1024)
    ws = torch.empty(pr.pr_hist_workspace_size(K, 1024), dtype=torch.uint8, device="cuda")
    rho = torch.empty((K, 1024), dtype=torch.float64, device="cuda")
    for _ in range(2):
        pr.pr_hist_restrict(x, None, N, K, grid, rho, ws)
        torch.cuda.synchronize()
    rt = torch.roll(rho, 5, dims=1).contiguous()
    mws = torch.empty(pr.pr_hist_match_workspace_size(N, K, 1024), dtype=torch.uint8, device="cuda")
    xo, yo, wo = torch.empty_like(x), torch.empty_like(y), torch.empty_like(x)
    for kind in (pr.PR_M_MARGINAL, pr.PR_M_RESAMPLE):
        for _ in range(2):
            pr.pr_hist_match(kind, rt, rho, N, K, 1, grid, x, y, None, N, xo, yo, wo, mws, seed=0, instance=0,
                             t_first=1)
            torch.cuda.synchronize()


def chem():
    """The chemical-reaction fine propagator on the workload of Table 1:
    P = 1e5, N = 20 slices of T = 40 (dt = 1e-3), all slices in one launch."""
    n, k, s_total, dt = 100_000, 20, 40_000, 1e-3
    c = pr.Chem()
    x0 = torch.empty(n, dtype=torch.float64, device="cuda")
    y0 = torch.empty(n, dtype=torch.float64, device="cuda")
    pr.pr_chem_init_ensemble(c, 0, 0, n, x0, y0)
    x, y = x0.repeat(k, 1).contiguous(), y0.repeat(k, 1).contiguous()
    sched = pr.Schedule(s_total, k, dt)
    for _ in range(2):
        xs, ys = x.clone(), y.clone()
        pr.pr_chem_fine_propagate(c, sched, 0, 0, n, 0, k, xs, ys)
        torch.cuda.synchronize()


def adjoint():
    """Differentiated form: P = 2^20, 1e4 steps of dt = 1e-4 (lambda = 1,
    eps = 0.1, beta = 2), checkpoints every 256 steps, the four observables'
    seed vectors, one reverse sweep for all four."""
    n, s_total, dt, every = 2 ** 20, 10_000, 1e-4, 256
    sde = pr.Sde(lam=1.0, eps=0.1, beta=2.0)
    sched = pr.Schedule(s_total, 1, dt)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    ck = torch.empty(((s_total + every - 1) // every, 2, n), dtype=torch.float64, device="cuda")
    obs = torch.empty(4, dtype=torch.float64, device="cuda")
    seeds = torch.empty((4, n), dtype=torch.float64, device="cuda")
    wso = torch.empty(pr.pr_observables_workspace_size(n), dtype=torch.uint8, device="cuda")
    jac = torch.empty((4, 4), dtype=torch.float64, device="cuda")
    wsa = torch.empty(pr.pr_adjoint_workspace_size(n, every, 4), dtype=torch.uint8, device="cuda")
    for _ in range(2):
        pr.pr_init_ensemble(sde, 0, 0, n, x, y)
        pr.pr_fine_checkpoint(sde, sched, 0, 0, n, x, y, ck, every)
        pr.pr_observables(x, n, [0.1, 0.5, 0.9], obs, wso, seed_x=seeds)
        pr.pr_fine_adjoint(sde, sched, 0, 0, n, ck, every, seeds, 4, jac, wsa)
        torch.cuda.synchronize()


def batch():
    """Batched form as the benchmark runs it: 256 instances drawn from seed
    0 (eps log-uniform in [1e-3, 1e-1], lambda in [0.5, 2], P in 2^12..2^18,
    8..64 slices, dt = eps/20, T = 2, 200 cells, 100 levels; the fine launch
    shape autotuned); creation runs the zeroth iteration, then one iteration
    in batched launches and two as graph replays."""
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        draw = torch.empty((256, 4), dtype=torch.float64, device="cuda")
        pr.pr_draw_instances(0, 256, draw)
        sdes, scheds, ns = [], [], []
        for eps, lam, lg, k in draw.cpu().numpy():
            dt = eps / 20
            s_total = int(round(2.0 / dt))
            sdes.append(pr.Sde(lam=float(lam), eps=float(eps), beta=2.0))
            scheds.append(pr.Schedule(s_total, int(k), 2.0 / s_total))
            ns.append(2 ** int(lg))
        h = pr.pr_parareal_batch_create(sdes, scheds, ns, pr.Grid(n_cells=200, n_q=100), 0, flags=pr.PR_AUTOTUNE)
        try:
            print("batch: created", flush=True)
            pr.pr_parareal_batch_iterate(h, 1, pr.PR_LAUNCH_BATCHED)
            torch.cuda.synchronize()
            print("batch: batched iteration done", flush=True)
            pr.pr_parareal_batch_iterate(h, 2, pr.PR_LAUNCH_GRAPH)
            torch.cuda.synchronize()
            print("batch: graph iterations done", flush=True)
        finally:
            pr.pr_parareal_batch_destroy(h)


if __name__ == "__main__":
    group = sys.argv[1] if len(sys.argv) > 1 else "fine"
    {"fine": fine, "restrict": restrict, "match": match, "copy": copy, "hist": hist, "chem": chem, "adjoint": adjoint,
     "batch": batch}[group]()
    print(f"profile_workload {group}: done", flush=True)
