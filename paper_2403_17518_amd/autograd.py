"""Differentiation through the propagator (torch.autograd).

* ``forward_model(v)``: d = F(v). Its backward is the adjoint J^T applied to
  the incoming data gradient, computed by ``born_mig`` (paper section 2.3
  eq. 13: the adjoint of the Born operator), which recomputes the forward
  wavefield from stored D^n history or checkpoints instead of keeping
  thousands of time levels alive in autograd.
* ``misfit(v, d_obs)``: phi = 1/2 ||F(v) - d_obs||^2 (section 2.1 eq. 2).
  Forward and gradient come from one ``fwi_gradient`` call; the backward
  only scales the stored gradient.

Both take a :class:`~paper_2403_17518_amd.ops.FwiContext` (or use the
default context of the tensor's device). Gradients are with respect to v
itself: a grid that asks for the relative-perturbation operator is run with
the velocity parametrisation here.
"""
from __future__ import annotations

from dataclasses import replace

import torch

from . import ops


def _ctx(fctx, v):
    return fctx if fctx is not None else ops.default_context(v.device.index or 0)


def _velocity(grid):
    return replace(grid, relative=False) if getattr(grid, "relative", False) else grid


class _ForwardModel(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, grid, acq, fctx):
        d = fctx.fwi_forward(grid, acq, v.detach().contiguous())
        ctx.save_for_backward(v)
        ctx.grid, ctx.acq, ctx.fctx = grid, acq, fctx
        return d

    @staticmethod
    def backward(ctx, grad_d):
        (v,) = ctx.saved_tensors
        g = None
        if ctx.needs_input_grad[0]:
            g = ctx.fctx.born_mig(ctx.grid, ctx.acq, v.detach().contiguous(),
                                  grad_d.detach().contiguous().to(torch.float32))
        return g, None, None, None


class _Misfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, d_obs, grid, acq, fctx):
        g, phi, _ = fctx.fwi_gradient(grid, acq, v.detach().contiguous(),
                                      d_obs.detach().contiguous(), want_misfit=True)
        ctx.save_for_backward(g)
        ctx.d_obs_needs_grad = d_obs.requires_grad
        return torch.tensor(phi, dtype=torch.float64, device=v.device)

    @staticmethod
    def backward(ctx, grad_phi):
        (g,) = ctx.saved_tensors
        gv = (grad_phi.to(torch.float32) * g) if ctx.needs_input_grad[0] else None
        if ctx.needs_input_grad[1]:
            raise NotImplementedError("misfit(): gradient with respect to d_obs is not provided; "
                                      "use forward_model() and an explicit loss instead")
        return gv, None, None, None, None


def forward_model(v: torch.Tensor, grid, acq, fctx: ops.FwiContext | None = None) -> torch.Tensor:
    """d = F(v), differentiable in v (backward = J^T via the adjoint sweep)."""
    return _ForwardModel.apply(v, _velocity(grid), acq, _ctx(fctx, v))


def misfit(v: torch.Tensor, d_obs: torch.Tensor, grid, acq,
           fctx: ops.FwiContext | None = None) -> torch.Tensor:
    """phi = 1/2 ||F(v) - d_obs||^2 as a float64 scalar, differentiable in v."""
    return _Misfit.apply(v, d_obs, _velocity(grid), acq, _ctx(fctx, v))
