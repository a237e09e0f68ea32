"""Differentiable collocation: D and atom centres -> level densities.

``collocate(gpw, D, coords)`` returns the level densities rho_l(D; R) of the
plan's system and records a backward that uses the library's own kernels
(Sec. III.B, Alg. 3 for the centre derivatives):

  dL/dD      = eval_mat(g_l / w_l)       (the adjoint of eval_rho in D)
  dL/dR_A    = eval_grad(D, g_l / w_l)   (d/dR_A sum_l w_l <g_l / w_l, rho_l>)

for an upstream gradient g_l = dL/drho_l.  The plan is built for one
geometry: ``coords`` must hold the plan's atom positions (it only carries
the gradient), and a new geometry needs a new plan.
"""
from __future__ import annotations

import numpy as np
import torch


class GPWCollocate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, D, coords, gpw):
        ref = torch.as_tensor(gpw.coords, dtype=torch.float64)
        if tuple(coords.shape) != tuple(ref.shape) or not torch.equal(coords.detach().cpu(), ref):
            raise ValueError("coords differ from the plan's geometry; build a plan for them")
        rho = gpw.rho(D.detach().contiguous())
        ctx.gpw = gpw
        ctx.coords_device = coords.device
        ctx.save_for_backward(D)
        return tuple(rho)

    @staticmethod
    def backward(ctx, *g_rho):
        (D,) = ctx.saved_tensors
        gpw = ctx.gpw
        V = []
        for l, g in enumerate(g_rho):
            if g is None:
                g = torch.zeros(tuple(gpw.meshes[l]), dtype=torch.float64, device=D.device)
            V.append((g / gpw.weights[l]).contiguous())
        dD = gpw.mat(V) if ctx.needs_input_grad[0] else None
        dR = None
        if ctx.needs_input_grad[1]:
            dR = gpw.grad(D.detach().contiguous(), V).to(ctx.coords_device)
        return dD, dR, None


def collocate(gpw, D, coords):
    """Level densities as a tuple of tensors, differentiable in D and coords."""
    return GPWCollocate.apply(D, coords, gpw)
