"""torch.autograd front end of the adjoint path.

TransmittedProbability(theta) = P_T(psi_N) with psi_N = S^N psi_0 and
V = sum_j theta_j G_j.  Forward runs dl_expand, dl_step and dl_observables;
it keeps only psi_N.  Backward rebuilds the trajectory backwards with the
fused reverse step (dl_seed_adjoint, dl_grad_step) and projects dL/dV on the
parameters (dl_project); no intermediate state is stored.
"""
from __future__ import annotations

import torch


class TransmittedProbability(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, plan, psi0, G, nsteps, x_b):
        if theta.dtype != torch.float64:
            raise TypeError("theta must be float64")
        V = torch.empty(plan.tshape[:-1], dtype=torch.float64, device=psi0.device)
        plan.expand(G, theta.detach().contiguous(), V)
        psi = psi0.detach().clone()
        plan.step(psi, V, int(nsteps))
        obs = plan.observables(psi, float(x_b))
        ctx.plan, ctx.nsteps, ctx.x_b = plan, int(nsteps), float(x_b)
        ctx.save_for_backward(psi, V, G)
        return torch.tensor(obs[4], dtype=torch.float64, device=psi0.device)

    @staticmethod
    def backward(ctx, grad_out):
        psiN, V, G = ctx.saved_tensors
        plan = ctx.plan
        psi = psiN.clone()
        lam = torch.empty_like(psi)
        Q = torch.empty(plan.tshape[:-1], dtype=torch.float64, device=psi.device)
        plan.seed_adjoint(psi, ctx.x_b, lam, Q)
        plan.grad_step(psi, lam, V, Q, ctx.nsteps)
        g = torch.empty(G.shape[0], dtype=torch.float64, device=psi.device)
        plan.project(Q, G, g)
        return grad_out * g, None, None, None, None, None


def transmitted_probability(theta, plan, psi0, G, nsteps, x_b):
    return TransmittedProbability.apply(theta, plan, psi0, G, nsteps, x_b)
