"""torch.autograd front end of the adjoint path.

TransmittedProbability(theta) = P_T(psi_N) with psi_N = S^N psi_0 and
V = sum_j theta_j G_j.  Forward runs dl_expand, dl_step and dl_observables;
it keeps only psi_N (and a reference to the caller's psi_0).  Backward
rebuilds the trajectory backwards with the fused reverse step
(dl_seed_adjoint, dl_grad_step) and projects dL/dV on the parameters
(dl_project); no intermediate state is stored.

The rebuild applies S^H, which inverts a step exactly on a periodic box, and
with zero walls only while no probability has crossed a wall.  Backward
therefore compares the norm of the rebuilt psi_0 with that of the true one
(both from dl_observables) and warns (ReconstructionWarning) when they differ
by more than rounding: the gradient is then not that of the forward run.
"""
from __future__ import annotations

import warnings

import torch


class ReconstructionWarning(UserWarning):
    """The backward sweep did not return to psi_0 (probability left through a
    zero wall during the forward run); the gradient is unreliable."""


# relative norm mismatch tolerated between the rebuilt and the true psi_0:
# rounding of the forward and reverse sweeps (FP64 state: ~1e-15 per step;
# FP32 state: ~1e-7 per step, random-walk accumulated)
RECON_TOL = {torch.complex128: 1e-9, torch.complex64: 1e-4}


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
        ctx.save_for_backward(psi, V, G, psi0.detach())
        return torch.tensor(obs[4], dtype=torch.float64, device=psi0.device)

    @staticmethod
    def backward(ctx, grad_out):
        psiN, V, G, psi0 = ctx.saved_tensors
        plan = ctx.plan
        psi = psiN.clone()
        lam = torch.empty_like(psi)
        Q = torch.empty(plan.tshape[:-1], dtype=torch.float64, device=psi.device)
        plan.seed_adjoint(psi, ctx.x_b, lam, Q)
        plan.grad_step(psi, lam, V, Q, ctx.nsteps)
        g = torch.empty(G.shape[0], dtype=torch.float64, device=psi.device)
        plan.project(Q, G, g)
        n_true = plan.observables(psi0, ctx.x_b)[0]
        n_rebuilt = plan.observables(psi, ctx.x_b)[0]
        tol = RECON_TOL.get(psi.dtype, 1e-4)
        if abs(n_rebuilt - n_true) > tol * abs(n_true):
            warnings.warn(f"the reverse sweep rebuilt psi_0 with norm {n_rebuilt:.12g} instead "
                          f"of {n_true:.12g}: probability left the box through a zero wall, so "
                          "S^H no longer inverts the steps and the gradient is unreliable "
                          "(use a periodic box or a larger one)", ReconstructionWarning,
                          stacklevel=2)
        return grad_out * g, None, None, None, None, None


def transmitted_probability(theta, plan, psi0, G, nsteps, x_b):
    return TransmittedProbability.apply(theta, plan, psi0, G, nsteps, x_b)
