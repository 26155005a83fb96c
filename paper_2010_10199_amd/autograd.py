"""Differentiable grouped transform: torch.autograd.Function over the HIP library.

forward:   f = F(X) fhat                              (gt_plan_trafo)
backward:  grad_fhat = F(X)^H grad_f                  (gt_plan_adjoint; F is C-linear)
           grad_x[v, j] = Re(conj(d f_v / d x_{v,j}) grad_f_v)   (gt_plan_node_grad)
with grad_f the conjugate-Wirtinger gradient torch passes to backward.  Batched over R
right-hand sides on shared nodes or over ragged datasets (offsets), one plan per call.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import lib


def _prec(dtype: torch.dtype):
    if dtype == torch.complex64:
        return lib.GT_C64, torch.float32
    if dtype == torch.complex128:
        return lib.GT_C128, torch.float64
    raise TypeError("fhat must be complex64 or complex128")


class GroupedTrafo(torch.autograd.Function):
    @staticmethod
    def forward(ctx, fhat, x, d, ds, N, offsets, m, sigma):
        code, rdt = _prec(fhat.dtype)
        if x.dtype != rdt:
            raise TypeError("x must have the real dtype matching fhat")
        if not (fhat.is_cuda and x.is_cuda):
            raise RuntimeError("grouped transform runs on the GPU only")
        fhat_c = fhat.detach().contiguous()
        x_c = x.detach().contiguous()
        R = fhat_c.shape[0] if fhat_c.dim() == 2 else 1
        Mx = x_c.shape[0]
        prob, keep = lib.make_problem(d, ds, N, M=Mx if offsets is None else 0, R=R, dtype=code, m=m, sigma=sigma,
                                      offsets=offsets)
        plan = lib.Plan(prob, x_c, keepalive=keep)
        nout = R * Mx if offsets is None else Mx
        f = torch.empty(nout, dtype=fhat.dtype, device=fhat.device)
        plan.trafo(fhat_c, f)
        ctx.plan = plan
        ctx.save_for_backward(fhat_c)
        ctx.shape_fhat = fhat.shape
        ctx.shape_x = x.shape
        f = f.view(R, Mx) if (offsets is None and fhat.dim() == 2) else f
        return f

    @staticmethod
    def backward(ctx, gf):
        (fhat_c,) = ctx.saved_tensors
        plan = ctx.plan
        g = gf.contiguous()
        grad_fhat = grad_x = None
        if ctx.needs_input_grad[0]:
            grad_fhat = torch.empty(ctx.shape_fhat, dtype=fhat_c.dtype, device=fhat_c.device)
            plan.adjoint(g, grad_fhat)
        if ctx.needs_input_grad[1]:
            rdt = torch.float32 if fhat_c.dtype == torch.complex64 else torch.float64
            grad_x = torch.empty(ctx.shape_x, dtype=rdt, device=fhat_c.device)
            plan.node_grad(fhat_c, g, grad_x)
        return grad_fhat, grad_x, None, None, None, None, None, None


def grouped_trafo(fhat: torch.Tensor, x: torch.Tensor, d: int, ds: int, N: Sequence[int],
                  offsets: Optional[Sequence[int]] = None, m: int = 0, sigma: float = 0.0) -> torch.Tensor:
    """Differentiable f = F(X) fhat.  fhat: (R, |I|) or (|I|,) complex; x: (Mtot, d) real."""
    return GroupedTrafo.apply(fhat, x, int(d), int(ds), tuple(int(v) for v in N),
                              None if offsets is None else tuple(int(v) for v in offsets), int(m), float(sigma))
