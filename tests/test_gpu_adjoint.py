"""GPU parity of the pathwise adjoint: the reverse sweep on the GPU against the
oracle's forward-mode tangents (a different algorithm) for the same seed
vectors, against common-random-number central differences of the GPU's own
forward runs, and through the torch.autograd binding."""
import sys

import numpy as np
import pytest

import paper_1912_09240_amd as pr
from oracle import particles as OP
from oracle import restrict as OR

pytestmark = pytest.mark.gpu

ALPHA = (0.1, 0.5, 0.9)


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


def _forward(torch, theta, n, S, dt, every, seed=0):
    lam, eps, beta, c3 = theta
    sde = pr.Sde(lam=lam, eps=eps, beta=beta, c3=c3)
    sched = pr.Schedule(S, 1, dt)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    pr.pr_init_ensemble(sde, seed, 0, n, x, y)
    ck = torch.empty(((S + every - 1) // every, 2, n), dtype=torch.float64, device="cuda")
    pr.pr_fine_checkpoint(sde, sched, seed, 0, n, x, y, ck, every)
    obs = torch.empty(1 + len(ALPHA), dtype=torch.float64, device="cuda")
    seeds = torch.empty((1 + len(ALPHA), n), dtype=torch.float64, device="cuda")
    ws = torch.empty(pr.pr_observables_workspace_size(n), dtype=torch.uint8, device="cuda")
    pr.pr_observables(x, n, ALPHA, obs, ws, seed_x=seeds)
    return sde, sched, x, y, ck, obs, seeds


@pytest.mark.parametrize("n,S,every", [(4097, 1003, 256), (1000, 300, 64), (65, 17, 256), (1000, 300, 8),
                                       (513, 101, 5)])
def test_adjoint_matches_oracle_tangents(torch_dev, n, S, every):
    torch = torch_dev
    _say(f"adjoint vs tangents n={n} S={S} every={every}")
    theta = (1.0, 0.1, 2.0, 1.0)
    dt = 1e-3
    sde, sched, x, y, ck, obs, seeds = _forward(torch, theta, n, S, dt, every)
    k = seeds.shape[0]
    jac = torch.empty((k, 4), dtype=torch.float64, device="cuda")
    ws = torch.empty(pr.pr_adjoint_workspace_size(n, every, k), dtype=torch.uint8, device="cuda")
    pr.pr_fine_adjoint(sde, sched, 0, 0, n, ck, every, seeds, k, jac, ws)
    torch.cuda.synchronize()
    so = OP.Sde(lam=1.0, eps=0.1, beta=2.0, c3=1.0)
    xo, yo, dx, dy = OP.em_tangent(so, 0, 0, n, S, dt)
    assert np.abs(x.cpu().numpy() - xo).max() < 1e-12
    # observables
    ob = obs.cpu().numpy()
    assert abs(ob[0] - OR.moments(xo)[1]) < 1e-10 * abs(ob[0])
    xs = np.sort(xo)
    for a, al in enumerate(ALPHA):
        assert abs(ob[1 + a] - OR.hazen_at(xs, al)[0]) < 1e-10
    # vector-Jacobian products of the same seeds
    sd = seeds.cpu().numpy()
    ref = sd @ dx.T  # [k][4]
    got = jac.cpu().numpy()
    scale = np.abs(ref).max(axis=1, keepdims=True) + 1e-300
    assert np.all(np.abs(got - ref) <= 1e-10 * scale), (got, ref)


def test_adjoint_crn_finite_differences(torch_dev):
    """Central differences of mean X_T^2 with common random numbers
    (h = 1e-5) against the adjoint."""
    torch = torch_dev
    _say("adjoint vs CRN FD")
    n, S, dt, every, h = 16384, 500, 1e-3, 256, 1e-5
    theta = [1.0, 0.1, 2.0, 1.0]
    sde, sched, x, y, ck, obs, seeds = _forward(torch, theta, n, S, dt, every)
    jac = torch.empty((4, 4), dtype=torch.float64, device="cuda")
    ws = torch.empty(pr.pr_adjoint_workspace_size(n, every, 4), dtype=torch.uint8, device="cuda")
    pr.pr_fine_adjoint(sde, sched, 0, 0, n, ck, every, seeds, 4, jac, ws)
    g = jac.cpu().numpy()[0]
    for t in range(4):
        vals = []
        for sgn in (1, -1):
            th = list(theta)
            th[t] += sgn * h
            vals.append(_forward(torch, th, n, S, dt, every)[5].cpu().numpy()[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[t]) < 1e-6 * max(1.0, abs(g[t])), (t, fd, g[t])


def test_autograd_binding(torch_dev):
    torch = torch_dev
    _say("autograd")
    from paper_1912_09240_amd.autograd import ParamGrad
    cfg = dict(n=8192, S=400, dt=1e-3, every=128)
    theta = torch.tensor([1.0, 0.1, 2.0, 1.0], dtype=torch.float64, device="cuda", requires_grad=True)
    obs = ParamGrad.apply(theta, cfg)
    w = torch.tensor([1.0, -0.5, 0.25, 2.0], dtype=torch.float64, device="cuda")
    (gt,) = torch.autograd.grad((obs * w).sum(), theta)
    sde, sched, x, y, ck, obs2, seeds = _forward(torch, (1.0, 0.1, 2.0, 1.0), 8192, 400, 1e-3, 128)
    jac = torch.empty((4, 4), dtype=torch.float64, device="cuda")
    ws = torch.empty(pr.pr_adjoint_workspace_size(8192, 128, 4), dtype=torch.uint8, device="cuda")
    pr.pr_fine_adjoint(sde, sched, 0, 0, 8192, ck, 128, seeds, 4, jac, ws)
    assert torch.equal(obs.detach(), obs2)
    assert torch.allclose(gt, w @ jac, rtol=1e-12, atol=0)


def test_checkpoint_forward_is_the_fine_propagator_bitwise(torch_dev):
    """The checkpointed forward steps with the fine propagator's own
    Euler-Maruyama step: every checkpoint and the final state equal
    pr_fine_propagate over the same steps bit for bit (here the slices of a
    schedule whose slice bounds are the checkpoint steps)."""
    torch = torch_dev
    n, every, nck = 5000, 64, 7
    S = every * nck
    _say(f"checkpoint forward vs fine propagate n={n} S={S}")
    sde = pr.Sde(lam=1.0, eps=0.1, beta=2.0, c3=1.0)
    dt = 1e-3
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    pr.pr_init_ensemble(sde, 5, 2, n, x, y)
    x2, y2 = x.clone(), y.clone()
    ck = torch.empty((nck, 2, n), dtype=torch.float64, device="cuda")
    pr.pr_fine_checkpoint(sde, pr.Schedule(S, 1, dt), 5, 2, n, x, y, ck, every)
    sched = pr.Schedule(S, nck, dt)
    for s in range(nck):
        assert torch.equal(ck[s, 0], x2) and torch.equal(ck[s, 1], y2), s
        pr.pr_fine_propagate(sde, sched, 5, 2, n, s, 1, x2, y2)
    torch.cuda.synchronize()
    assert torch.equal(x, x2) and torch.equal(y, y2)


def test_adjoint_full_size_on_a_particle_subset(torch_dev):
    """The differentiated form at its full size (P = 2^20, 1e4 steps of
    1e-4, checkpoints every 256 steps, 40 segments) with four seed vectors
    that are non-zero on particles 0..1023 only: the reverse sweep of the
    whole ensemble equals the oracle's forward-mode tangents of those 1024
    particles (counter-based noise makes the subset exact) to 1e-10
    relative, the initial law's dependence on beta included."""
    torch = torch_dev
    n, S, dt, every, m = 2 ** 20, 10_000, 1e-4, 256, 1024
    _say(f"adjoint full size n={n} S={S} subset={m}")
    sde = pr.Sde(lam=1.0, eps=0.1, beta=2.0, c3=1.0)
    sched = pr.Schedule(S, 1, dt)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    pr.pr_init_ensemble(sde, 0, 0, n, x, y)
    ck = torch.empty(((S + every - 1) // every, 2, n), dtype=torch.float64, device="cuda")
    pr.pr_fine_checkpoint(sde, sched, 0, 0, n, x, y, ck, every)
    rng = np.random.default_rng(41)
    sx = np.zeros((4, n))
    sy = np.zeros((4, n))
    sx[:, :m] = rng.normal(0.0, 1.0, (4, m))
    sy[:, :m] = rng.normal(0.0, 1.0, (4, m))
    sy[0, :m] = 0.0  # one seed on the slow variable alone
    jac = torch.empty((4, 4), dtype=torch.float64, device="cuda")
    ws = torch.empty(pr.pr_adjoint_workspace_size(n, every, 4), dtype=torch.uint8, device="cuda")
    pr.pr_fine_adjoint(sde, sched, 0, 0, n, ck, every, torch.from_numpy(sx).cuda(), 4, jac, ws,
                       seed_y=torch.from_numpy(sy).cuda())
    torch.cuda.synchronize()
    xo, yo, dx, dy = OP.em_tangent(OP.Sde(lam=1.0, eps=0.1, beta=2.0, c3=1.0), 0, 0, m, S, dt)
    assert np.abs(x.cpu().numpy()[:m] - xo).max() < 1e-12
    ref = sx[:, :m] @ dx.T + sy[:, :m] @ dy.T
    got = jac.cpu().numpy()
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert np.all(scale > 0.0)
    assert np.all(np.abs(got - ref) <= 1e-10 * scale), (got, ref)
