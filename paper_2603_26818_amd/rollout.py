"""Differentiable PFC rollout: gradients of a loss on psi(T) with respect to psi0 and r.

Forward: ``nsteps`` semi-implicit steps (pfc_step) from psi0, keeping (psi, state) every
``checkpoint_every`` steps.  Backward: for each segment, newest first, replay the segment from its
checkpoint keeping every psi^n (the step is deterministic, so the replay reproduces the forward
bit for bit), then apply the transpose of each step's Jacobian (pfc_step_backward) from the last
step of the segment to the first.  pfc_step_backward also accumulates dL/dr in an FP64 device
scalar.  All arithmetic runs in the library's kernels; this module only orders the calls.
"""
from __future__ import annotations

import torch

from ._binding import Plan


class PFCRollout(torch.autograd.Function):
    """psi_T = PFCRollout.apply(psi0, r, plan, nsteps, checkpoint_every).

    psi0: real field on the plan's device (plan dtype), r: 0-d float64 tensor (the undercooling).
    The plan's dt and operator are fixed; its r is set from ``r`` for the run."""

    @staticmethod
    def forward(ctx, psi0, r, plan: Plan, nsteps: int, checkpoint_every: int = 50):
        if checkpoint_every < 1:
            raise ValueError("checkpoint_every must be >= 1")
        rv = float(r.detach().cpu()) if isinstance(r, torch.Tensor) else float(r)
        dt = plan.dt
        plan.set_params(rv, dt)
        psi = psi0.detach().clone().contiguous()
        state = plan.state_init(psi)
        ckpts = []
        done = 0
        while done < nsteps:
            seg = min(checkpoint_every, nsteps - done)
            ckpts.append((psi.clone(), state.clone(), seg))
            plan.step(psi, state, seg)
            done += seg
        ctx.plan = plan
        ctx.rv = rv
        ctx.ckpts = ckpts
        return psi

    @staticmethod
    def backward(ctx, grad_out):
        plan: Plan = ctx.plan
        plan.set_params(ctx.rv, plan.dt)
        lam = grad_out.detach().to(plan.real_dtype).contiguous().clone()
        dLdr = torch.zeros(1, dtype=torch.float64, device=plan.device)
        for psi_c, state_c, seg in reversed(ctx.ckpts):
            traj = [psi_c]
            psi = psi_c.clone()
            state = state_c.clone()
            for _ in range(seg):
                plan.step(psi, state, 1)
                traj.append(psi.clone())
            for n in range(seg - 1, -1, -1):
                plan.step_backward(traj[n], traj[n + 1], lam, lambda_n=lam, dLdr=dLdr)
            del traj
        ctx.ckpts = None
        grad_r = dLdr.reshape(()).cpu() if ctx.needs_input_grad[1] else None
        return lam, grad_r, None, None, None


def loss_and_grad(plan: Plan, psi0: torch.Tensor, r: float, target: torch.Tensor, nsteps: int,
                  checkpoint_every: int = 50):
    """L = sum (psi_T - target)^2 and (dL/dpsi0, dL/dr) through PFCRollout."""
    x = psi0.detach().clone().requires_grad_(True)
    rt = torch.tensor(float(r), dtype=torch.float64, requires_grad=True)
    psi_T = PFCRollout.apply(x, rt, plan, nsteps, checkpoint_every)
    diff = psi_T - target
    L = torch.sum(diff.double() * diff.double())
    L.backward()
    return float(L.detach()), x.grad.detach(), float(rt.grad)
