"""Benchmark of the micro-macro parareal hot path on one MI355X.

Workload (the large configuration of the method): the 2-D slow-fast SDE
dX = -(X^3 - X + lambda (X - Y)) dt + sqrt(2/beta) dW1,
dY = -(1/eps)(Y - X) dt + sqrt(2/(beta eps)) dW2, lambda = 1, beta = 2,
eps = 0.01; P = 2^20 FP64 particles, dt = 1e-4, T = 10 (S = 1e5 steps) in
N = 64 slices, coarse grid of 1024 cells on [-3, 3], 100 quantile levels.
Synthetic, Philox-seeded inputs (seed 0).

A step is one parareal iteration k -> k+1 over the whole hot path: fine
propagation of all 64 slices in one launch, restriction (sort, ranks,
knots) of the fine results, coarse propagation of every slice, the serial
quantile-iterator chain, matching of every slice, and the knots of the new
states with their RMS error to the serial fine run.  value = P * S / (time
of one step): fine particle-steps per second of the whole iteration.

The roofline object is for the dominant kernel (the fine propagator): its
duration is the summed HIP-event time of its launches over the timed steps,
recorded on the stream it runs on.  The CPU baseline is the plain oracle
running one iteration of the same workload on a bounded particle sample.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (fwd+adjoint) and parareal sweep time vs plain, same tol"
WORKLOAD = dict(lam=1.0, beta=2.0, eps=0.01, n=2 ** 20, dt=1e-4, T=10.0, K=64, cells=1024, nq=100, seed=0)

# VALU instructions of one FP64 particle-step (d = 1) on gfx950, the
# instruction stream the method needs with no address arithmetic, spills or
# loop control on the vector unit: Philox4x32-10 with the particle index as
# the only lane-varying counter word (15 lane-varying 32x32->64 products and
# 17 xor: 32), the Box-Muller pair from table lookups in LDS (u from bit
# fields 2, -2 ln u from a 1024-cell table 12, sqrt 7, sin/cos of the angle
# 14, two products 2: 37) and the Euler-Maruyama update (10): 79, counted on
# isolated builds of each part.  The figure changes only with the method's
# arithmetic, so that the fraction moves with speed alone.
VALU_OPS_PER_STEP = 79
# What the compiled kernel issues per particle-step by SQ_INSTS_VALU (154.06
# per wave-step of two particles), valid while the sources hash to
# FINE_SOURCES_SHA256: two fewer than the frozen figure, since the slow part's
# cubic and linear terms are one polynomial in x (update 9) and the step loop,
# unrolled twice with a 32-bit counter on the scalar unit, has no copies of
# the state and no vector compare.  Its rate against the peak is the issue
# utilisation.
KERNEL_VALU_PER_STEP = 154.06 / 2
# MI355X: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz = VALU lane-ops/s
VALU_PEAK = 256 * 64 * 2.4e9
HBM_PEAK = 8.0e12  # B/s
# FP64 vector peak of MI355X (256 CUs x 128 FP64 flop per clock x 2.4 GHz)
FP64_PEAK = 78.6e12
# FP64 flops of the Euler-Maruyama update of one particle-step (d = 1),
# eq. (EMx)/(EMy) with dt folded into the coefficients: slow part 11
# (d = x - y, x^2, (-dt c3) x^2 and four fused multiply-adds of two flops:
# the cubic, linear and coupling terms and the noise), fast part 4 (two fused
# multiply-adds, d shared).  The normals' own arithmetic is not counted.  The
# kernel now takes the cubic and linear terms as one polynomial in x (14
# flops); the figure stays, like VALU_OPS_PER_STEP.
FP64_FLOP_PER_STEP = 15

# HBM bytes of one launch of the fine kernel (all 64 slices) from two
# rocprofv3 counter passes, FETCH_SIZE x 2.0 (the factor a 1 GiB copy needs)
# + WRITE_SIZE, valid while the kernel's sources hash to FINE_SOURCES_SHA256.
FINE_TRAFFIC_BYTES = (524440 * 2 + 1048576) * 1024
FINE_SOURCES_SHA256 = "ae8a2ccd719189505a28721d0c149e5f8e6851200a8ae949f78d752ad4ff2273"
FINE_SOURCES = ["pr_fine.hip", "pr_fine_dev.hpp", "pr_internal.hpp", "pr_normal.hpp", "pr_fastmath.hpp",
                "pr_noise_tables.inc"]


def fine_sources_sha256():
    h = hashlib.sha256()
    for f in FINE_SOURCES:
        with open(os.path.join(ROOT, "paper_1912_09240_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=8192, help="particles in the oracle's sample")
    ap.add_argument("--flags", type=int, default=0, help="parareal flags (1 reuse coarse, 2 skip converged)")
    ap.add_argument("--detail", default="bench_detail.json",
                    help="file for the full measurements (empty: none)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(n_sample):
    """One parareal iteration of the workload by the oracle, on particles
    0..n_sample-1 (counter-based noise makes the sample exact), on the
    process's OpenMP threads; then on one thread, on an eighth of the
    sample."""
    from oracle import coarse as OC
    from oracle import iterate as OI
    from oracle import particles as OP
    w = WORKLOAD
    sde = OP.Sde(lam=w["lam"], eps=w["eps"], beta=w["beta"])

    def one_iteration(n):
        po, hp = OI.micmac_parareal(sde, w["seed"], 0, n, w["T"], w["dt"], w["K"], OC.Grid(w["cells"]), w["nq"])
        t0 = time.perf_counter()
        po.iterate()
        return n * hp["S"], time.perf_counter() - t0

    steps, t = one_iteration(n_sample)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = dict(value=steps / t, unit="particle-steps/s", cores=threads, kind="oracle",
               sample=f"one parareal iteration (fine propagation of all {w['K']} slices, restriction, coarse "
                      f"propagation, quantile-iterator chain, matching) of the large workload on particles "
                      f"0..{n_sample - 1}; {t:.2f} s on {threads} OpenMP threads",
               cpu_model=_cpu_model(), nproc=os.cpu_count())
    set_threads = getattr(OP.lib(), "omp_set_num_threads", None)
    if set_threads is not None and threads > 1:
        set_threads.argtypes = [ctypes.c_int]
        set_threads(1)
        n1 = max(64, n_sample // 8)
        steps1, t1 = one_iteration(n1)
        set_threads(threads)
        out["one_thread"] = dict(value=steps1 / t1, sample=f"particles 0..{n1 - 1}, {t1:.2f} s on one OpenMP thread")
    return out


ADJOINT = dict(lam=1.0, beta=2.0, eps=0.1, c3=1.0, n=2 ** 20, S=10_000, dt=1e-4, every=256, seed=0,
               alpha=(0.1, 0.5, 0.9))
# VALU instructions of one particle-step of forward + reverse sweep with four
# seed vectors and checkpoints every 256 steps: the forward step (79, as the
# fine propagator), the reverse sweep's two replays of it (2 x 79) and the
# reverse recursion (the step's Jacobian and parameter derivatives, 29, and
# per seed vector four gradient updates and the 2 x 2 transposed Jacobian
# product, 10, for four vectors 40: 69): 306
ADJ_OPS_PER_STEP = 79 + 2 * 79 + 69


def adjoint_measure(torch, pr):
    """Differentiated form: P = 2^20, 1e4 steps of dt = 1e-4, checkpoints every
    256 steps, observables mean X_T^2 and the 0.1/0.5/0.9 quantiles, all four
    rows of the Jacobian w.r.t. (lambda, eps, beta, c3) in one reverse sweep.
    Times (HIP events on the current stream): forward with checkpoints,
    observables, reverse sweep; and a plain forward for the comparison with
    8 common-random-number finite-difference runs."""
    a = ADJOINT
    n, S, dt, every = a["n"], a["S"], a["dt"], a["every"]
    sde = pr.Sde(lam=a["lam"], eps=a["eps"], beta=a["beta"], c3=a["c3"])
    sched = pr.Schedule(S, 1, dt)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    ck = torch.empty(((S + every - 1) // every, 2, n), dtype=torch.float64, device="cuda")
    k = 1 + len(a["alpha"])
    obs = torch.empty(k, dtype=torch.float64, device="cuda")
    seeds = torch.empty((k, n), dtype=torch.float64, device="cuda")
    wso = torch.empty(pr.pr_observables_workspace_size(n), dtype=torch.uint8, device="cuda")
    jac = torch.empty((k, 4), dtype=torch.float64, device="cuda")
    wsa = torch.empty(pr.pr_adjoint_workspace_size(n, every, k), dtype=torch.uint8, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    for rep in range(2):  # second repetition is the measured one
        pr.pr_init_ensemble(sde, a["seed"], 0, n, x, y)
        ev[0].record()
        pr.pr_fine_checkpoint(sde, sched, a["seed"], 0, n, x, y, ck, every)
        ev[1].record()
        pr.pr_observables(x, n, list(a["alpha"]), obs, wso, seed_x=seeds)
        ev[2].record()
        pr.pr_fine_adjoint(sde, sched, a["seed"], 0, n, ck, every, seeds, k, jac, wsa)
        ev[3].record()
        pr.pr_init_ensemble(sde, a["seed"], 0, n, x, y)
        ev[4].record()
        pr.pr_fine_propagate(sde, sched, a["seed"], 0, n, 0, 1, x, y)
        ev[5].record()
        torch.cuda.synchronize()
    t_fwd = ev[0].elapsed_time(ev[1]) / 1e3
    t_obs = ev[1].elapsed_time(ev[2]) / 1e3
    t_adj = ev[2].elapsed_time(ev[3]) / 1e3
    t_plain = ev[4].elapsed_time(ev[5]) / 1e3
    total = t_fwd + t_obs + t_adj
    jac256 = jac.clone()
    # memory for time: checkpoints every 8 steps are the reverse sweep's tape
    # starts, which drops its first recomputation (1250 x 2 x 2^20 doubles)
    del ck, wsa
    torch.cuda.empty_cache()
    e8 = 8
    ck8 = torch.empty(((S + e8 - 1) // e8, 2, n), dtype=torch.float64, device="cuda")
    ws8 = torch.empty(pr.pr_adjoint_workspace_size(n, e8, k), dtype=torch.uint8, device="cuda")
    for rep in range(2):
        pr.pr_init_ensemble(sde, a["seed"], 0, n, x, y)
        ev[0].record()
        pr.pr_fine_checkpoint(sde, sched, a["seed"], 0, n, x, y, ck8, e8)
        ev[1].record()
        pr.pr_observables(x, n, list(a["alpha"]), obs, wso, seed_x=seeds)
        ev[2].record()
        pr.pr_fine_adjoint(sde, sched, a["seed"], 0, n, ck8, e8, seeds, k, jac, ws8)
        ev[3].record()
        torch.cuda.synchronize()
    t_fwd8 = ev[0].elapsed_time(ev[1]) / 1e3
    t_adj8 = ev[2].elapsed_time(ev[3]) / 1e3
    jac_rel = float(((jac - jac256).abs().max(dim=1).values / jac256.abs().max(dim=1).values).max())
    every8 = dict(checkpoint_bytes=ck8.numel() * 8, forward_ckpt_s=t_fwd8, reverse_s=t_adj8,
                  reverse_over_forward=t_adj8 / t_fwd8, jacobian_rel_diff_vs_every256=jac_rel)
    del ck8, ws8
    torch.cuda.empty_cache()
    return dict(workload="adjoint of the 2-D SDE (lambda=1, beta=2, eps=0.1), P=2^20 FP64, 1e4 steps of dt=1e-4, "
                         "checkpoints every 256 steps, observables mean X_T^2 and quantiles 0.1/0.5/0.9, "
                         "4x4 Jacobian w.r.t. (lambda, eps, beta, c3) in one reverse sweep",
                fwd_plus_adjoint_particle_steps_per_s=n * S / total,
                valu_frac=ADJ_OPS_PER_STEP * (n * S / total) / VALU_PEAK, ops_per_particle_step=ADJ_OPS_PER_STEP,
                forward_ckpt_s=t_fwd, observables_s=t_obs,
                reverse_s=t_adj, plain_forward_s=t_plain, reverse_over_forward=t_adj / t_fwd,
                ratio_to_8_crn_fd_forwards=total / (8 * t_plain),
                ckpt_every_8=every8,
                jacobian=jac256.cpu().tolist(), observables=obs.cpu().tolist())


BATCH = dict(count=256, T=2.0, beta=2.0, cells=200, nq=100, seed=0)


def batched_measure(torch, pr):
    """Batched form: 256 instances of the 2-D SDE with eps log-uniform in
    [1e-3, 1e-1], lambda ~ U(0.5, 2), P in {2^12..2^18}, N in {8..64} slices,
    dt = eps/20, T = 2 (drawn from the seed), coarse grid 200 cells, 100
    levels.  Two handles of the same batch run the same number of
    iterations: one as batched launches and hipGraph replays, the other
    instance by instance (the plain launch pattern).  Their knots of every
    state of every instance are then compared bit for bit, so the sweep times
    are compared at the same quantile error.  Device time per iteration from
    HIP events, and the device time of all four iterations of each handle
    (to the final iteration; the graph capture is host work before the first
    timed replay)."""
    b = BATCH
    stream = torch.cuda.Stream()  # graph capture needs a non-default stream
    with torch.cuda.stream(stream):
        draw = torch.empty((b["count"], 4), dtype=torch.float64, device="cuda")
        pr.pr_draw_instances(b["seed"], b["count"], draw)
        d = draw.cpu().numpy()
        sdes, scheds, ns = [], [], []
        for eps, lam, lg, K in d:
            dt = eps / 20
            S = int(round(b["T"] / dt))
            sdes.append(pr.Sde(lam=float(lam), eps=float(eps), beta=b["beta"]))
            scheds.append(pr.Schedule(S, int(K), b["T"] / S))
            ns.append(2 ** int(lg))
        grid = pr.Grid(n_cells=b["cells"], n_q=b["nq"])
        rows = sum(sc.n_slices + 1 for sc in scheds)

        def knots(h):
            out = torch.empty((rows, b["nq"] + 1), dtype=torch.float64, device="cuda")
            r = 0
            for i, sc in enumerate(scheds):
                for t in range(sc.n_slices + 1):
                    pr.pr_parareal_batch_state(h, i, t, q=out[r])
                    r += 1
            return out

        t0 = time.perf_counter()
        h = pr.pr_parareal_batch_create(sdes, scheds, ns, grid, b["seed"], flags=pr.PR_AUTOTUNE)
        t_create = time.perf_counter() - t0
        try:
            info = pr.pr_parareal_batch_info(h)
            ms_first = pr.pr_parareal_batch_iterate(h, 1, pr.PR_LAUNCH_GRAPH, timed=True)  # captures first
            ms_graph = pr.pr_parareal_batch_iterate(h, 2, pr.PR_LAUNCH_GRAPH, timed=True) / 2
            ms_batched = pr.pr_parareal_batch_iterate(h, 1, pr.PR_LAUNCH_BATCHED, timed=True)
            qa = knots(h)
        finally:
            pr.pr_parareal_batch_destroy(h)
        h = pr.pr_parareal_batch_create(sdes, scheds, ns, grid, b["seed"], flags=pr.PR_AUTOTUNE)
        try:
            ms_plain3 = pr.pr_parareal_batch_iterate(h, 3, pr.PR_LAUNCH_PER_INSTANCE, timed=True)
            ms_plain = pr.pr_parareal_batch_iterate(h, 1, pr.PR_LAUNCH_PER_INSTANCE, timed=True)
            qb = knots(h)
        finally:
            pr.pr_parareal_batch_destroy(h)
        same = bool(torch.equal(qa, qb))
    w = info["particle_steps"]
    return dict(workload="256 instances of the 2-D SDE, eps log-uniform [1e-3, 1e-1], lambda U(0.5, 2), "
                         "P in 2^12..2^18, N in 8..64 slices, dt = eps/20, T = 2, 200 cells, 100 levels",
                fine_particle_steps_per_iteration=w, work_units=info["units"],
                tuned_block=info["block"], tuned_particles_per_thread=info["ppt"],
                tuned_split_sort=info["split_sort"],
                sweep_ms_graph=ms_graph, sweep_ms_batched=ms_batched, sweep_ms_per_instance=ms_plain,
                particle_steps_per_s_graph=w / (ms_graph / 1e3),
                particle_steps_per_s_per_instance=w / (ms_plain / 1e3),
                speedup_vs_per_instance=ms_plain / ms_graph, create_s=t_create,
                same_quantile_error=same, iterations_compared=4,
                to_final_ms_batched=ms_first + 2 * ms_graph + ms_batched,
                to_final_ms_per_instance=ms_plain3 + ms_plain,
                # the sweep against its floor: the fine particle-steps at the
                # VALU issue peak (the restriction, chains and matching count
                # as overhead here)
                sweep_floor_ms=1e3 * VALU_OPS_PER_STEP * w / VALU_PEAK,
                sweep_floor_frac_graph=(1e3 * VALU_OPS_PER_STEP * w / VALU_PEAK) / ms_graph)


HIGHDIM = dict(d=32, n=2 ** 20, dt=1e-4, T=5.0, K=32, eps=0.01, beta=2.0, lam=1.0, seed=0)


HIST_COMBOS = [("quantile", "marginal"), ("quantile", "reweight"), ("quantile", "resample"),
               ("quantile", "resample_det"), ("add", "resample"), ("mult", "resample"), ("rot", "resample")]


def hist_measure(torch, pr, w, n, K, S, dt):
    """Histogram-state iterations (Sec. 4 iterators, Sec. 5 matchings) on the
    large workload: one warm-up and one timed iteration per combination with
    the phase times, and the L2 error of the states' histograms to the
    serial fine run after the timed iteration (device time from HIP events
    recorded by the driver)."""
    its = dict(add=pr.PR_J_ADD, mult=pr.PR_J_MULT, rot=pr.PR_J_ROT, quantile=pr.PR_J_QUANTILE)
    mts = dict(marginal=pr.PR_M_MARGINAL, reweight=pr.PR_M_REWEIGHT, resample=pr.PR_M_RESAMPLE,
               resample_det=pr.PR_M_RESAMPLE_DET)
    sde = pr.Sde(lam=w["lam"], eps=w["eps"], beta=w["beta"])
    sched = pr.Schedule(S, K, dt)
    grid = pr.Grid(n_cells=w["cells"], n_q=w["nq"])
    I = w["cells"]
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    pr.pr_init_ensemble(sde, w["seed"], 0, n, x, y)
    ref = torch.empty((K + 1, I), dtype=torch.float64, device="cuda")
    ws = torch.empty(pr.pr_hist_workspace_size(1, I), dtype=torch.uint8, device="cuda")
    pr.pr_hist_restrict(x, None, n, 1, grid, ref[0], ws)
    for s_ in range(K):
        pr.pr_fine_propagate(sde, sched, w["seed"], 0, n, s_, 1, x, y)
        pr.pr_hist_restrict(x, None, n, 1, grid, ref[s_ + 1], ws)
    out = {}
    for it, mt in HIST_COMBOS:
        h = pr.pr_parareal_hist_create(sde, sched, grid, w["seed"], 0, n, its[it], mts[mt], flags=pr.PR_PROFILE)
        try:
            pr.pr_parareal_hist_iterate(h, 1)
            p0, i0 = pr.pr_parareal_hist_profile(h)
            err = np.zeros(2)
            pr.pr_parareal_hist_iterate(h, 1, rho_ref=ref, err_out=err)
            p1, i1 = pr.pr_parareal_hist_profile(h)
        finally:
            pr.pr_parareal_hist_destroy(h)
        ph = {k: p1[k] - p0[k] for k in p1}
        rest = ph["restrict_fine"] / 1e3
        out[f"{it}+{mt}"] = dict(ms_per_iteration=sum(v for k, v in ph.items() if k != "restrict_new"),
                                 phases_ms=ph, l2_error_at_T=float(err[0]), l2_error_max=float(err[1]),
                                 restrict_fine_GBps=n * K * (16 if mt == "reweight" else 8) / rest / 1e9)
    return dict(workload="histogram states (1024 cells on [-3, 3]) of the large workload: P=2^20, 64 slices, "
                         "1e5 steps of dt=1e-4; iterator + matching per entry; errors after two iterations",
                combos=out)


# VALU instructions of one particle-step of the chemical-reaction fine kernel:
# Philox 32, the Box-Muller logarithm and angle without its square root (31),
# the drift and diffusion of the reaction network, two square roots of the
# amplitude times -2 ln u and the update (35): the compiled two-particle loop
# issued 197 per step; unrolled twice with its 32-bit counter on the scalar
# unit it issues 194 (the figure stays, so the fraction moves with speed).
CHEM_VALU_PER_STEP = 98


def chem_measure(torch, pr):
    """The paper's own workload (Sec. 6, Table 1): chemical-reaction system,
    P = 1e5 particles, N = 20 slices of T = 40 (dt = 1e-3, 40000 steps),
    grid [0, 600] with h = 1 (600 cells).  For every iterator x matching
    combination, K = 20 iterations with the L2 error of the slow variable's
    histogram after each one against a serial run with ten times the
    particles (its first P particles are the parareal ensemble, so the error
    of a serial P-particle run is the floor).  Device times from HIP events
    recorded by the driver."""
    its = dict(add=pr.PR_J_ADD, mult=pr.PR_J_MULT, rot=pr.PR_J_ROT, quantile=pr.PR_J_QUANTILE)
    mts = dict(marginal=pr.PR_M_MARGINAL, reweight=pr.PR_M_REWEIGHT, resample=pr.PR_M_RESAMPLE,
               resample_det=pr.PR_M_RESAMPLE_DET)
    n, K, S, dt, I, seed = 100_000, 20, 40_000, 1e-3, 600, 0
    nr = 10 * n
    chem, sched = pr.Chem(), pr.Schedule(S, K, dt)
    grid = pr.Grid(n_cells=I, x_lo=0.0, x_hi=600.0)
    x = torch.empty(nr, dtype=torch.float64, device="cuda")
    y = torch.empty(nr, dtype=torch.float64, device="cuda")
    pr.pr_chem_init_ensemble(chem, seed, 0, nr, x, y)
    ref = torch.empty((K + 1, I), dtype=torch.float64, device="cuda")
    own = torch.empty((K + 1, I), dtype=torch.float64, device="cuda")
    ws = torch.empty(pr.pr_hist_workspace_size(1, I), dtype=torch.uint8, device="cuda")
    pr.pr_hist_restrict(x, None, nr, 1, grid, ref[0], ws)
    pr.pr_hist_restrict(x, None, n, 1, grid, own[0], ws)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    serial_ms = 0.0
    for s_ in range(K):
        ev[0].record()
        pr.pr_chem_fine_propagate(chem, sched, seed, 0, nr, s_, 1, x, y)
        ev[1].record()
        torch.cuda.synchronize()
        serial_ms += ev[0].elapsed_time(ev[1])
        pr.pr_hist_restrict(x, None, nr, 1, grid, ref[s_ + 1], ws)
        pr.pr_hist_restrict(x, None, n, 1, grid, own[s_ + 1], ws)
    floor = torch.sqrt(((own - ref) ** 2).sum(dim=1)).cpu().numpy()
    del x, y
    out = {}
    fine_ms = []
    for it in its:
        for mt in mts:
            log(f"chemical {it}+{mt}")
            h = pr.pr_parareal_hist_create_chem(chem, sched, grid, seed, 0, n, its[it], mts[mt], flags=pr.PR_PROFILE)
            try:
                err = np.zeros(2 * K)
                pr.pr_parareal_hist_iterate(h, K, rho_ref=ref, err_out=err)
                ph, iters = pr.pr_parareal_hist_profile(h)
            finally:
                pr.pr_parareal_hist_destroy(h)
            ph = {k: v / iters for k, v in ph.items()}
            fine_ms.append(ph["fine"])
            out[f"{it}+{mt}"] = dict(
                ms_per_iteration=sum(v for k, v in ph.items() if k != "restrict_new"), phases_ms=ph,
                l2_error_at_T=[float("%.4g" % e) for e in err[0::2]],
                l2_error_max=[float("%.4g" % e) for e in err[1::2]])
    fine = float(np.median(fine_ms))
    rate = n * S / (fine / 1e3)
    # Table 1 as printed (k3 = 0.666e-6): the fast variable's drift has one
    # root, near 7000, so the slow variable heads for k4 ybar / k5 far beyond
    # the experiment's grid [0, 600]; the same ensemble run over T = 40
    printed = pr.Chem(k=(60.0, 1.0, 4.8e-3, 0.666e-6, 0.833, 1.0))
    xp = torch.empty(n, dtype=torch.float64, device="cuda")
    yp = torch.empty(n, dtype=torch.float64, device="cuda")
    pr.pr_chem_init_ensemble(printed, seed, 0, n, xp, yp)
    pr.pr_chem_fine_propagate(printed, pr.Schedule(S, 1, dt), seed, 0, n, 0, 1, xp, yp)
    torch.cuda.synchronize()
    printed_k3 = dict(k3=0.666e-6, x_mean_at_T=float(xp.mean()), y_mean_at_T=float(yp.mean()),
                      fraction_x_beyond_600=float((xp > 600.0).double().mean()))
    del xp, yp
    return dict(printed_k3=printed_k3,
                workload="chemical-reaction system (Table 1: tau_x=25, eps=2.5e-2, k=(60, 1, 4.8e-3, 0.666e-5, "
                         "0.833, 1)), lognormal X0, Y0 (mean 100, sd 20), P=1e5, N=20, T=40, dt=1e-3, "
                         "600 cells on [0, 600]; K=20 iterations per iterator + matching; L2 histogram errors "
                         "after each iteration against a serial run with 1e6 particles",
                fine_ms=fine, fine_particle_steps_per_s=rate,
                fine_valu_frac=CHEM_VALU_PER_STEP * rate / VALU_PEAK,
                serial_fine_ms_1e6_particles=serial_ms,
                floor_l2_error_serial_1e5=[float("%.4g" % e) for e in floor],
                combos=out)


def advection_measure(torch, pr):
    """Linear-advection study (Sec. 6): fine model Fbar = x, Dbar = 1 on 800
    cells of [-8, 8], X0 ~ N(2, 1/4), T = 1 in N = 10 slices; coarse models
    with beta~ = 2 (underdiffusive), eps~ = 2 (wrong advection speed) and
    beta~ = 1/2 (overdiffusive).  For every iterator: the L2 error of the
    masses at T against the serial fine run after k = 0..5 iterations, and
    the device time of one iteration."""
    import scipy.stats as st
    I, K, T = 800, 10, 1.0
    grid = pr.Grid(n_cells=I, x_lo=-8.0, x_hi=8.0)
    sched = pr.Schedule(100 * K, K, T / (100 * K))
    edges = np.linspace(-8.0, 8.0, I + 1)
    c = st.norm.cdf(edges, loc=2.0, scale=0.5)
    r0 = np.diff(c)
    r0[0] += c[0]
    r0[-1] += 1.0 - c[-1]
    rho0 = torch.from_numpy(r0).cuda()
    its = dict(add=pr.PR_J_ADD, mult=pr.PR_J_MULT, rot=pr.PR_J_ROT, quantile=pr.PR_J_QUANTILE)
    hf = pr.pr_advection_coarse_create(1.0, 1.0, sched, grid)
    ref = torch.empty((K + 1, I), dtype=torch.float64, device="cuda")
    ref[0] = rho0
    out = {}
    try:
        # the serial fine run through the fine model's own exponentials
        hs = pr.pr_parareal_fp_create(hf, hf, grid, rho0, pr.PR_J_ADD)
        try:
            for t in range(K + 1):
                pr.pr_parareal_fp_state(hs, t, ref[t])
        finally:
            pr.pr_parareal_fp_destroy(hs)
        for name, (ec, bc) in dict(underdiffusive=(1.0, 2.0), advection=(2.0, 1.0),
                                    overdiffusive=(1.0, 0.5)).items():
            hc = pr.pr_advection_coarse_create(ec, bc, sched, grid)
            try:
                row = {}
                for it, kind in its.items():
                    h = pr.pr_parareal_fp_create(hf, hc, grid, rho0, kind)
                    try:
                        rho = torch.empty(I, dtype=torch.float64, device="cuda")
                        pr.pr_parareal_fp_state(h, K, rho)
                        errs = [float(torch.sqrt(((rho - ref[K]) ** 2).sum()))]
                        e = np.zeros(2 * 5)
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        pr.pr_parareal_fp_iterate(h, 5, rho_ref=ref, err_out=e)
                        ms = (time.perf_counter() - t0) * 1e3 / 5
                        errs += [float(v) for v in e[0::2]]
                    finally:
                        pr.pr_parareal_fp_destroy(h)
                    row[it] = dict(l2_error_at_T=[float("%.3g" % v) for v in errs], ms_per_iteration=ms)
                out[name] = dict(coarse=dict(eps=ec, beta=bc), iterators=row)
            finally:
                pr.pr_coarse_destroy(hc)
    finally:
        pr.pr_coarse_destroy(hf)
    return dict(workload="linear advection: Fbar = x/eps, Dbar = 1/beta, eps = beta = 1, 800 cells on [-8, 8], "
                         "X0 ~ N(2, 1/4), T = 1, N = 10; errors after k = 0..5 iterations",
                models=out)


def highdim_measure(torch, pr):
    """Fast part in R^32 (dY_i = -(1/eps)(Y_i - a_i X) dt + ..., a_i from the
    seed): one fine sweep of all 32 slices (P = 2^20, 5e4 steps of 1e-4) in
    FP64 and in FP32 stepping, from the initial ensemble in every slice.
    FP32 error stated as the knot difference to the FP64 run (the FP64 path
    matches the oracle per particle to 1e-12)."""
    h = HIGHDIM
    n, K, d = h["n"], h["K"], h["d"]
    S = int(round(h["T"] / h["dt"]))
    a = torch.empty(d, dtype=torch.float64, device="cuda")
    pr.pr_draw_coupling(h["seed"], 0, d, a)
    out = {}
    knots = {}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for prec, dtype in ((pr.PR_F64, torch.float64), (pr.PR_F32, torch.float32)):
        sde = pr.Sde(lam=h["lam"], eps=h["eps"], beta=h["beta"], d=d, a=a, precision=prec)
        x0 = torch.empty(n, dtype=dtype, device="cuda")
        y0 = torch.empty((d, n), dtype=dtype, device="cuda")
        pr.pr_init_ensemble(sde, h["seed"], 0, n, x0, y0)
        x = x0.repeat(K, 1).contiguous()
        y = y0.repeat(K, 1, 1).contiguous()
        del y0
        ev[0].record()
        pr.pr_fine_propagate(sde, pr.Schedule(S, K, h["T"] / S), h["seed"], 0, n, 0, K, x, y)
        ev[1].record()
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1]) / 1e3
        xs = x[K - 1].to(torch.float64).contiguous()
        q = torch.empty(101, dtype=torch.float64, device="cuda")
        ws = torch.empty(pr.pr_restrict_workspace_size(n, 1), dtype=torch.uint8, device="cuda")
        pr.pr_restrict_quantiles(xs, pr.PR_F64, n, 1, 100, q, ws)
        knots[prec] = q.cpu().numpy()
        out["fp64" if prec == pr.PR_F64 else "fp32"] = dict(sweep_s=t, particle_steps_per_s=n * S / t)
        del x, y, x0
        torch.cuda.empty_cache()
    err = knots[pr.PR_F32] - knots[pr.PR_F64]
    out["fp32_knot_error_vs_fp64"] = dict(max_abs_interior=float(np.abs(err[1:-1]).max()),
                                          rms=float(np.sqrt(np.mean(err ** 2))))
    out["workload"] = ("fast part in R^32, a_i ~ U(0.5, 1.5) from the seed, eps = 0.01, P = 2^20, "
                       "dt = 1e-4, T = 5 in 32 slices, one sweep of all slices")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU sharding of the slices is described in the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1912_09240_amd as pr

    w = WORKLOAD
    S = int(round(w["T"] / w["dt"]))
    dt = w["T"] / S
    n, K, nq = w["n"], w["K"], w["nq"]
    sde = pr.Sde(lam=w["lam"], eps=w["eps"], beta=w["beta"])
    sched = pr.Schedule(S, K, dt)
    grid = pr.Grid(n_cells=w["cells"], n_q=nq)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    # serial fine run: reference knots q_ref[t] for the error metric
    log("serial fine reference")
    t0 = time.perf_counter()
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    pr.pr_init_ensemble(sde, w["seed"], 0, n, x, y)
    qref = torch.empty((K + 1, nq + 1), dtype=torch.float64, device="cuda")
    ws = torch.empty(pr.pr_restrict_workspace_size(n, 1), dtype=torch.uint8, device="cuda")
    pr.pr_restrict_quantiles(x, pr.PR_F64, n, 1, nq, qref[0], ws)
    for s in range(K):
        pr.pr_fine_propagate(sde, sched, w["seed"], 0, n, s, 1, x, y)
        pr.pr_restrict_quantiles(x, pr.PR_F64, n, 1, nq, qref[s + 1], ws)
    torch.cuda.synchronize()
    t_serial = time.perf_counter() - t0
    del ws, x, y

    log("parareal create (zeroth iteration)")
    t0 = time.perf_counter()
    h = pr.pr_parareal_create(sde, sched, grid, w["seed"], 0, n, args.flags | pr.PR_PROFILE)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    errs = np.zeros(2 * (args.warmup + args.steps))
    try:
        for i in range(args.warmup):
            pr.pr_parareal_iterate(h, 1, q_ref=qref, err_out=errs[2 * i:])
            log(f"warmup iteration {i + 1} done")
        prof0, it0 = pr.pr_parareal_profile(h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            j = args.warmup + i
            pr.pr_parareal_iterate(h, 1, q_ref=qref, err_out=errs[2 * j:])
            log(f"timed iteration {i + 1} done")
        torch.cuda.synchronize()
        t_steps = time.perf_counter() - t0
        prof1, it1 = pr.pr_parareal_profile(h)
    finally:
        pr.pr_parareal_destroy(h)
    phases = {k: (prof1[k] - prof0[k]) / max(1, it1 - it0) for k in prof1}
    ms_step = 1e3 * t_steps / args.steps
    value = n * S / (t_steps / args.steps)

    fine_s = phases["fine"] / 1e3
    fine_rate = n * S / fine_s
    achieved = VALU_OPS_PER_STEP * fine_rate
    traffic = FINE_TRAFFIC_BYTES if fine_sources_sha256() == FINE_SOURCES_SHA256 else None
    roofline = dict(bound="alu", achieved=achieved / 1e12, peak=VALU_PEAK / 1e12, unit="Tops/s",
                    frac=achieved / VALU_PEAK, traffic=traffic,
                    traffic_algorithmic=n * K * 32,
                    kernel="fine_kernel<1,double,2> (all 64 slices, one launch)",
                    fine_ms=phases["fine"], fine_particle_steps_per_s=fine_rate,
                    ops_per_particle_step=VALU_OPS_PER_STEP,
                    kernel_ops_per_particle_step=KERNEL_VALU_PER_STEP if traffic is not None else None,
                    issue_frac=KERNEL_VALU_PER_STEP * fine_rate / VALU_PEAK if traffic is not None else None)

    # the whole iteration against its floor: the fine steps at the VALU issue
    # peak plus the algorithmic bytes of restriction (8 B key read + 4 B rank
    # write), matching (20 B) and the knots of the new states (8 B sorted key
    # read) per particle and slice at 8 TB/s; the serial chain and the coarse
    # step are latency and count as overhead
    floor_s = VALU_OPS_PER_STEP * n * S / VALU_PEAK + n * K * (12 + 20 + 8) / HBM_PEAK
    sweep_roofline = dict(floor_ms=1e3 * floor_s, measured_ms=ms_step, frac=1e3 * floor_s / ms_step,
                          basis=f"{VALU_OPS_PER_STEP} VALU instructions per particle-step at "
                                f"{VALU_PEAK / 1e12:.1f} T lane-instructions/s, 40 B per particle and slice at 8 TB/s")

    # the HBM-bound phases against the bytes the method must move per particle
    # and slice: the restriction's key read and rank write (12 B; a sort
    # moves several times that, and its counted bytes are in the profiles),
    # the matching's state read, rank read and state write (20 B), and the
    # sorted-key read behind the knots of the new states (8 B)
    hbm_phases = {}
    for name, per in (("restrict_fine", 12), ("match", 20), ("restrict_new", 8)):
        b = n * K * per
        t = phases[name] * 1e-3
        hbm_phases[name] = dict(bytes=b, ms=phases[name], achieved_gbs=b / t / 1e9, frac=b / t / HBM_PEAK)

    qerr_T = [float(errs[2 * i]) for i in range(args.warmup + args.steps)]
    qerr_max = [float(errs[2 * i + 1]) for i in range(args.warmup + args.steps)]
    config = dict(workload="slow-fast SDE, eps=0.01, P=2^20 FP64 particles, dt=1e-4, T=10 (1e5 steps), 64 slices, "
                           "1024-cell coarse grid, 100 quantile levels, one parareal iteration per step",
                  particles=n, fine_steps=S, slices=K, cells=w["cells"], quantile_levels=nq, flags=args.flags,
                  seed=w["seed"])
    detail = dict(metric=METRIC, value=value, unit="particle-steps/s", steps=args.steps, warmup=args.warmup,
                  ms_per_step=ms_step, config=config, roofline=roofline, sweep_roofline=sweep_roofline,
                  hbm_phases=hbm_phases, phases_ms=phases,
                  quantile_error=dict(at_T=qerr_T, max_over_slices=qerr_max),
                  serial_fine_s=t_serial, create_s=t_create)
    log("adjoint")
    detail["adjoint"] = adjoint_measure(torch, pr)
    log("batched instances")
    detail["batched"] = batched_measure(torch, pr)
    log("fast part in R^32")
    detail["high_dim"] = highdim_measure(torch, pr)
    log("histogram states")
    detail["hist_states"] = hist_measure(torch, pr, w, n, K, S, dt)
    log("chemical-reaction workload")
    detail["chemical"] = chem_measure(torch, pr)
    log("linear advection")
    detail["advection"] = advection_measure(torch, pr)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        detail["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    if args.detail:
        os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
        with open(args.detail, "w") as f:
            json.dump(detail, f, indent=1)
    line = summary_line(detail, args, config)
    text = json.dumps(line, separators=(",", ":"))
    assert len(text) <= 4096, f"summary line of {len(text)} bytes"
    print(text, flush=True)


def _sig(v, digits=4):
    return None if v is None else float(f"{v:.{digits}g}")


def summary_line(d, args, config):
    """The one JSON line of the run: the large workload's iteration rate with
    its roofline, the CPU baseline, and short summaries of the differentiated
    and batched forms (the full measurements are in the detail file)."""
    r = d["roofline"]
    line = dict(metric=d["metric"], value=_sig(d["value"], 6), unit=d["unit"], n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=_sig(d["ms_per_step"], 6), higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f64", data="synthetic (Philox-seeded, seed 0)",
                config=dict(workload=config["workload"], particles=config["particles"],
                            fine_steps=config["fine_steps"], slices=config["slices"], cells=config["cells"],
                            quantile_levels=config["quantile_levels"], flags=config["flags"]))
    line["roofline"] = dict(bound=r["bound"], achieved=_sig(r["achieved"]), peak=_sig(r["peak"]), unit=r["unit"],
                            frac=_sig(r["frac"]), traffic=r["traffic"], kernel=r["kernel"],
                            ops_per_particle_step=r["ops_per_particle_step"],
                            kernel_ops_per_particle_step=_sig(r.get("kernel_ops_per_particle_step")),
                            issue_frac=_sig(r.get("issue_frac")), fine_ms=_sig(r["fine_ms"]),
                            fp64_flop_per_particle_step=FP64_FLOP_PER_STEP,
                            fp64_tflops=_sig(FP64_FLOP_PER_STEP * r["fine_particle_steps_per_s"] / 1e12),
                            fp64_flop_frac=_sig(FP64_FLOP_PER_STEP * r["fine_particle_steps_per_s"] / FP64_PEAK))
    cb = d.get("cpu_baseline")
    if cb:
        line["cpu_baseline"] = dict(value=_sig(cb["value"]), unit=cb["unit"], cores=cb["cores"], kind=cb["kind"],
                                    sample=cb["sample"], cpu_model=cb.get("cpu_model"),
                                    one_thread_value=_sig(cb.get("one_thread", {}).get("value")))
    a = d["adjoint"]
    line["adjoint"] = {k: (_sig(v) if isinstance(v, float) else v) for k, v in a.items()
                       if k not in ("workload", "jacobian", "observables", "ckpt_every_8")}
    if "ckpt_every_8" in a:
        e8 = a["ckpt_every_8"]
        line["adjoint"]["ckpt_every_8"] = dict(reverse_over_forward=_sig(e8["reverse_over_forward"]),
                                               reverse_s=_sig(e8["reverse_s"]),
                                               checkpoint_bytes=e8["checkpoint_bytes"])
    b = d["batched"]
    line["batched"] = dict(sweep_ms_graph=_sig(b["sweep_ms_graph"]), sweep_ms_batched=_sig(b["sweep_ms_batched"]),
                           sweep_ms_per_instance=_sig(b["sweep_ms_per_instance"]),
                           speedup_vs_per_instance=_sig(b["speedup_vs_per_instance"]),
                           particle_steps_per_s_graph=_sig(b["particle_steps_per_s_graph"]),
                           same_quantile_error=b["same_quantile_error"], iterations_compared=b["iterations_compared"],
                           to_final_ms_batched=_sig(b.get("to_final_ms_batched")),
                           to_final_ms_per_instance=_sig(b.get("to_final_ms_per_instance")),
                           sweep_floor_frac_graph=_sig(b.get("sweep_floor_frac_graph")))
    line["sweep_roofline"] = dict(floor_ms=_sig(d["sweep_roofline"]["floor_ms"]),
                                  frac=_sig(d["sweep_roofline"]["frac"]))
    line["hbm_phases"] = {k: dict(ms=_sig(v["ms"]), frac=_sig(v["frac"])) for k, v in d["hbm_phases"].items()}
    line["quantile_error_at_T"] = [_sig(e, 3) for e in d["quantile_error"]["at_T"]]
    line["serial_fine_s"] = _sig(d["serial_fine_s"])
    line["detail"] = args.detail
    return line


if __name__ == "__main__":
    main()
