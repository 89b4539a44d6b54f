"""torch.autograd view of the hand-written adjoint: the swimmer's net
displacement as a differentiable function of (driving amplitude, phase lag,
spring stiffness)."""
from __future__ import annotations

import copy

import torch

from .sim import Sim


def _with_params(case, theta):
    c = copy.deepcopy(case)
    a, psi, k = (float(v) for v in theta)
    for d in c.drives:
        d.amplitude, d.phase_lag = a, psi
    for s in c.springs:
        s.k = k
    return c


class SwimmerDisplacement(torch.autograd.Function):
    """J(theta) = net x displacement of the swimmer's centroid after
    ``steps`` coupled steps from rest, theta = (amplitude, phase_lag, k).

    The forward runs the GPU step and its adjoint in one call of the C-ABI
    (lbm_adjoint, checkpoints every ``checkpoint_every`` steps); backward
    returns the stored gradient times the incoming one."""

    @staticmethod
    def forward(ctx, theta, case, steps, storage="f32", checkpoint_every=50, device="cuda:0"):
        sim = Sim(_with_params(case, theta.detach().cpu().tolist()), storage=storage, device=device)
        J, grad = sim.adjoint(steps, checkpoint_every)
        sim.close()
        ctx.save_for_backward(torch.tensor(grad, dtype=theta.dtype, device=theta.device))
        return torch.tensor(J, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None, None, None, None, None


def swimmer_displacement(theta, case, steps, storage="f32", checkpoint_every=50, device="cuda:0"):
    return SwimmerDisplacement.apply(theta, case, steps, storage, checkpoint_every, device)
