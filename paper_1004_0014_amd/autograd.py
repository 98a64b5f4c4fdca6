"""torch.autograd.Function over the hand-written forward and adjoint kernels.

PCRProject.apply(w, f0, grid, geom, model) = P W_{x(w)} f0: the cone-beam
projection (eq. (2)'s P) of the reference image f0 warped by the PCA
deformation x = mean + U w (eq. (1), eq. (2) constraint; pull-back warp of
sections 2.2-2.3).  The backward pass is the adjoint of section 2.2's
gradient, split by input:

    g        = P^T dp                      (backprojection)
    dL/dw_k  = sum_v g[v] (df/dx)[v] . u_k  (warp Jacobian, contraction)
    dL/df0   = W^T g                       (transpose of the warp)

With dp = 2 (p - a y - b) the w-gradient is the paper's 2 U^T (df/dx)^T P^T r.
Every step runs in the HIP library; w is a 1-D tensor of K values (any device,
read as host scalars), f0 a contiguous FP32 or FP64 device tensor [nz][ny][nx].
"""
from __future__ import annotations

import torch

from . import _lib


class PCRProject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, f0, grid, geom, model):
        if f0.dtype not in (torch.float32, torch.float64):
            raise ValueError("f0 must be float32 or float64 for differentiation")
        wl = [float(v) for v in w.detach().cpu().tolist()]
        f0c = f0.detach().contiguous()
        dvf = _lib.dvf_compose(grid, model, wl, compute=f0.dtype)
        f = _lib.warp_volume(grid, f0c, dvf)
        p = _lib.forward_project(grid, geom, f)
        ctx.save_for_backward(w.detach(), f0c, dvf)
        ctx.grid, ctx.geom, ctx.model = grid, geom, model
        return p

    @staticmethod
    def backward(ctx, dp):
        w, f0, dvf = ctx.saved_tensors
        g = _lib.backproject_residual(ctx.grid, ctx.geom, dp.detach().to(f0.dtype).contiguous())
        grad_w = grad_f0 = None
        if ctx.needs_input_grad[0]:
            wl = [float(v) for v in w.cpu().tolist()]
            gw = _lib.warp_contract(ctx.grid, ctx.model, f0, wl, g)
            grad_w = torch.tensor(gw, dtype=w.dtype, device=w.device)
        if ctx.needs_input_grad[1]:
            grad_f0 = _lib.warp_adjoint(ctx.grid, dvf, g)
        return grad_w, grad_f0, None, None, None


def project(w, f0, grid, geom, model):
    """Differentiable P W_{x(w)} f0."""
    return PCRProject.apply(w, f0, grid, geom, model)
