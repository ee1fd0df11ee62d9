"""torch.autograd.Function wrappers of the discrete adjoint (argument
marshalling only: the forward and reverse sweeps run in the HIP library).

* ``Rhs``: (h, hu, hv, b) -> R = dW/dt of the inviscid operator at that state
  and bathymetry; its backward is the library's reverse mode of R
  (``esdg_rhs_vjp``).
* ``GaugeMisfit``: (b, H0, hu0, hv0) -> gauge-misfit loss after nsteps fixed
  steps (LSRK(5,4) or SSPRK(3,3), the solver's integrator) from
  h(0) = H0 - b, hu(0) = hu0, hv(0) = hv0; its backward is the checkpointed
  reverse sweep (``esdg_adjoint_backward``).

Both set the solver's bathymetry and state (the solver is an argument, not a
differentiable input).  Inputs are contiguous float64 CUDA tensors of shape
[K, (N+1)^2] on the solver's device.
"""
from __future__ import annotations

import torch


class Rhs(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h, hu, hv, b, solver):
        solver.set_bathymetry(b)
        solver.set_state(h, hu, hv)
        ctx.solver = solver
        ctx.save_for_backward(h, hu, hv, b)
        return tuple(solver.rhs(device=True))

    @staticmethod
    def backward(ctx, gh, ghu, ghv):
        h, hu, hv, b = ctx.saved_tensors
        s = ctx.solver
        s.set_bathymetry(b)
        s.set_state(h, hu, hv)
        z = torch.zeros_like(h)
        lam = [g.contiguous() if g is not None else z for g in (gh, ghu, ghv)]
        wh, whu, whv, wb = s.rhs_vjp(*lam)
        return wh, whu, whv, wb, None


class GaugeMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, H0, hu0, hv0, solver, target, nsteps: int, dt: float, every: int):
        solver.set_bathymetry(b)
        solver.set_state((H0 - b).contiguous(), hu0, hv0)
        loss = solver.adjoint_forward(nsteps, dt, every, target)
        ctx.solver = solver
        return torch.tensor(loss, dtype=torch.float64, device=b.device)

    @staticmethod
    def backward(ctx, g):
        gb, gh0, ghu0, ghv0 = ctx.solver.adjoint_backward(seed=float(g), device=True)
        # h(0) = H0 - b: the initial state carries b too
        return gb - gh0, gh0, ghu0, ghv0, None, None, None, None, None


def gauge_misfit(solver, b, H0, hu0, hv0, target, nsteps: int, dt: float, every: int = 20):
    return GaugeMisfit.apply(b, H0, hu0, hv0, solver, target, nsteps, dt, every)
