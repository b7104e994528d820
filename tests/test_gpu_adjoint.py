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


@pytest.mark.parametrize("n,S,every", [(4097, 1003, 256), (1000, 300, 64), (65, 17, 256)])
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
