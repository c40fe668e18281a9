"""torch.autograd.Function over the HIP forward/backward kernels.

forward:  (y, theta) -> (f, E) with y the float32 SoA positions (3N,) in the
          handle's internal node order and theta a float64 (n_mat, 3)
          device tensor of (mu, kappa, w) per material slot (per cell, or
          per cell and region for a batch with material regions).
backward: (dL/df, dL/dE) -> (dL/dy, dL/dtheta) from cm_forces_backward:
          dL/dy is a Hessian-vector product of the energy minus dL/dE times
          the forces; dL/dtheta is exact (f is linear in mu1, mu2, kappa).
"""
from __future__ import annotations

import torch


class MRForces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, theta, batch):
        theta = theta.detach().to(torch.float64).contiguous()
        batch.set_params(theta[:, 0], theta[:, 1], theta[:, 2])
        f, E = batch.forces(y.detach().contiguous())
        ctx.batch = batch
        ctx.save_for_backward(y.detach(), theta)
        return f, E

    @staticmethod
    def backward(ctx, grad_f, grad_E):
        y, theta = ctx.saved_tensors
        batch = ctx.batch
        # the handle's parameters may have changed since forward
        batch.set_params(theta[:, 0], theta[:, 1], theta[:, 2])
        gf = grad_f.contiguous().float() if grad_f is not None else None
        gE = grad_E.contiguous().double() if grad_E is not None else None
        ybar, tb = batch.backward(y, gf, gE)
        return ybar, tb.view(-1, 3), None


def mr_forces(y, theta, batch):
    """Forces and per-cell energies with autograd support."""
    return MRForces.apply(y, theta, batch)
