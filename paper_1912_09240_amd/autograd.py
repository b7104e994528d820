"""torch.autograd binding of the pathwise adjoint.

ParamGrad.apply(theta) runs the fine propagator from the initial ensemble
with checkpoints (pr_fine_checkpoint) and returns the observables of the slow
variable at the final step (pr_observables): mean X_T^2 and the midpoint
quantiles at the requested levels.  Its backward runs one reverse sweep
(pr_fine_adjoint) for all observables at once and applies the incoming
gradient to the resulting Jacobian.  theta = (lambda, eps, beta, c3).
"""
import torch

import paper_1912_09240_amd as pr


class ParamGrad(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, cfg):
        lam, eps, beta, c3 = (float(v) for v in theta.detach().cpu().tolist())
        n, S, dt, every, seed = cfg["n"], cfg["S"], cfg["dt"], cfg.get("every", 256), cfg.get("seed", 0)
        alpha = list(cfg.get("alpha", (0.1, 0.5, 0.9)))
        sde = pr.Sde(lam=lam, eps=eps, beta=beta, c3=c3, c1=cfg.get("c1", -1.0))
        sched = pr.Schedule(S, 1, dt)
        dev = theta.device if theta.is_cuda else torch.device("cuda")
        x = torch.empty(n, dtype=torch.float64, device=dev)
        y = torch.empty(n, dtype=torch.float64, device=dev)
        pr.pr_init_ensemble(sde, seed, 0, n, x, y)
        n_ck = (S + every - 1) // every
        ckpt = torch.empty((n_ck, 2, n), dtype=torch.float64, device=dev)
        pr.pr_fine_checkpoint(sde, sched, seed, 0, n, x, y, ckpt, every)
        k = 1 + len(alpha)
        obs = torch.empty(k, dtype=torch.float64, device=dev)
        seeds = torch.empty((k, n), dtype=torch.float64, device=dev)
        ws = torch.empty(pr.pr_observables_workspace_size(n), dtype=torch.uint8, device=dev)
        pr.pr_observables(x, n, alpha, obs, ws, seed_x=seeds)
        ctx.save_for_backward(ckpt, seeds)
        ctx.cfg = (sde, sched, seed, n, every, k)
        return obs.to(theta.device)

    @staticmethod
    def backward(ctx, grad_obs):
        ckpt, seeds = ctx.saved_tensors
        sde, sched, seed, n, every, k = ctx.cfg
        jac = torch.empty((k, 4), dtype=torch.float64, device=ckpt.device)
        ws = torch.empty(pr.pr_adjoint_workspace_size(n, every, k), dtype=torch.uint8, device=ckpt.device)
        pr.pr_fine_adjoint(sde, sched, seed, 0, n, ckpt, every, seeds, k, jac, ws, from_initial=True)
        g = grad_obs.to(jac.device, torch.float64) @ jac
        return g.to(grad_obs.device), None
