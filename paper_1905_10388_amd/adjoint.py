"""Gradient of the final kinetic energy with respect to the initial b grid:
a torch.autograd.Function over the HIP forward steps and their discrete
adjoint, with checkpointed recomputation.

Forward: X^0 = IC(b_grid), K multistep steps, J = KE(X^K); a checkpoint of
(X, history, step counters) is kept every `checkpoint` steps.  Backward: for
each segment, last first, restore its checkpoint, recompute the segment's
states, and reverse its steps with stau_adjoint_step; finally map the state
adjoint through the adjoint of the initial-condition map.
"""
from __future__ import annotations

import torch


def _forward(solver, b_grid, dt, steps, checkpoint):
    solver.initial_state(b_grid)
    ckpts = {}
    for n in range(steps):
        if n % checkpoint == 0:
            ckpts[n] = solver.snapshot()
        solver.step(dt)
    return solver.kinetic_energy(), ckpts


def _reverse(solver, dt, steps, checkpoint, ckpts, X_final):
    Xbar = solver.kinetic_energy_adjoint(X_final)
    _, hbar = solver.new_adjoint_state()
    for start in sorted(ckpts, reverse=True):
        end = min(start + checkpoint, steps)
        solver.restore(ckpts[start])
        seg = []
        for _ in range(start, end):
            seg.append((solver.X.clone(), solver.iteration, solver.dt_prev))
            solver.step(dt)
        for X_prev, it, dtp in reversed(seg):
            solver.adjoint_step(X_prev, it, dt, dtp, Xbar, hbar)
    return solver.initial_state_adjoint(Xbar)


def kinetic_energy_and_gradient(solver, b_grid, dt: float, steps: int, checkpoint: int = 20):
    """(J, dJ/d b_grid) without autograd bookkeeping."""
    J, ckpts = _forward(solver, b_grid, dt, steps, checkpoint)
    return J, _reverse(solver, dt, steps, checkpoint, ckpts, solver.X.clone())


class FinalKineticEnergy(torch.autograd.Function):
    """J = KE(X^K) as a differentiable function of the b grid tensor."""

    @staticmethod
    def forward(ctx, b_grid, solver, dt, steps, checkpoint):
        J, ckpts = _forward(solver, b_grid, dt, steps, checkpoint)
        # the final state of this forward pass seeds the reverse sweep, so
        # stepping the solver between forward and backward does not change it
        ctx.solver, ctx.dt, ctx.steps, ctx.checkpoint, ctx.ckpts = solver, dt, steps, checkpoint, ckpts
        ctx.X_final = solver.X.clone()
        ctx.b_dtype, ctx.b_device = b_grid.dtype, b_grid.device
        return torch.tensor(J, dtype=torch.float64, device=b_grid.device)

    @staticmethod
    def backward(ctx, gJ):
        g = _reverse(ctx.solver, ctx.dt, ctx.steps, ctx.checkpoint, ctx.ckpts, ctx.X_final)
        g = g.to(device=ctx.b_device, dtype=ctx.b_dtype)
        return gJ.to(device=ctx.b_device, dtype=ctx.b_dtype) * g, None, None, None, None


def final_kinetic_energy(b_grid, solver, dt: float, steps: int, checkpoint: int = 20):
    return FinalKineticEnergy.apply(b_grid, solver, dt, steps, checkpoint)
