"""Differentiable grouped transform: torch.autograd.Function over the HIP library.

forward:   f = F(X) fhat                              (gt_plan_trafo)
backward:  grad_fhat = F(X)^H grad_f                  (gt_plan_adjoint; F is C-linear)
           grad_x[v, j] = Re(conj(d f_v / d x_{v,j}) grad_f_v)   (gt_plan_node_grad)
with grad_f the conjugate-Wirtinger gradient torch passes to backward.  Batched over R
right-hand sides on shared nodes or over ragged datasets (offsets), one plan per call;
GroupedTrafoFixedNodes keeps one plan for nodes that do not change (coefficient gradients),
GroupedTrafoMovingNodes one plan whose nodes it moves in place on every call (both gradients).
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


class _TrafoMoving(torch.autograd.Function):
    """f = F(X) fhat on an owner's plan after moving its nodes to x; backward gives both
    gradients.  The owner's node version at the forward is checked in the backward."""

    @staticmethod
    def forward(ctx, fhat, x, owner):
        fhat_c = fhat.detach().contiguous()
        owner._set_nodes(x)
        f = torch.empty(owner.nout, dtype=fhat.dtype, device=fhat.device)
        owner.plan.trafo(fhat_c, f)
        ctx.owner = owner
        ctx.version = owner.version
        ctx.save_for_backward(fhat_c)
        ctx.shape_fhat, ctx.shape_x = fhat.shape, x.shape
        return f.view(owner.R, -1) if (owner.offsets is None and fhat.dim() == 2) else f

    @staticmethod
    def backward(ctx, gf):
        (fhat_c,) = ctx.saved_tensors
        owner = ctx.owner
        if owner.version != ctx.version:
            raise RuntimeError("GroupedTrafoMovingNodes: the nodes moved again before this backward ran "
                               "(run each call's backward before the next call)")
        g = gf.contiguous()
        grad_fhat = grad_x = None
        if ctx.needs_input_grad[0]:
            grad_fhat = torch.empty(ctx.shape_fhat, dtype=fhat_c.dtype, device=fhat_c.device)
            owner.plan.adjoint(g, grad_fhat)
        if ctx.needs_input_grad[1]:
            rdt = torch.float32 if fhat_c.dtype == torch.complex64 else torch.float64
            grad_x = torch.empty(ctx.shape_x, dtype=rdt, device=fhat_c.device)
            owner.plan.node_grad(fhat_c, g, grad_x)
        return grad_fhat, grad_x, None


class GroupedTrafoMovingNodes:
    """Differentiable f = F(X) fhat with gradients for fhat and the nodes, for nodes that change
    between calls (descent on the nodes): one plan is built for the first nodes and every
    later call moves its nodes in place (gt_plan_update_nodes: device re-binning, no new plan).
    The node count, datasets, bandwidths and precision are fixed at construction.  Each call's
    backward must run before the next call (the plan holds one node set); a backward that
    finds the nodes moved since its forward raises.

    x0: (Mtot, d) real CUDA tensor; calls take (fhat, x) as grouped_trafo does.  tune=True times
    the plan's launch forms on the first nodes (gt_plan_tune, on the current stream) and keeps
    them for the later nodes."""

    def __init__(self, x0: torch.Tensor, d: int, ds: int, N: Sequence[int], R: int = 1,
                 offsets: Optional[Sequence[int]] = None, m: int = 0, sigma: float = 0.0, tune: bool = False):
        if not x0.is_cuda:
            raise RuntimeError("grouped transform runs on the GPU only")
        code = lib.GT_C64 if x0.dtype == torch.float32 else lib.GT_C128 if x0.dtype == torch.float64 else None
        if code is None:
            raise TypeError("x must be float32 or float64")
        self.offsets = None if offsets is None else tuple(int(v) for v in offsets)
        self.R = int(R) if offsets is None else len(self.offsets) - 1
        self.shape = tuple(x0.shape)
        self.xdtype = x0.dtype
        x_c = x0.detach().contiguous()
        Mx = x_c.shape[0]
        prob, keep = lib.make_problem(d, ds, N, M=Mx if offsets is None else 0, R=self.R, dtype=code, m=m,
                                      sigma=sigma, offsets=self.offsets)
        self.plan = lib.Plan(prob, x_c, keepalive=keep)
        self.tuning = self.plan.tune(torch.cuda.current_stream().cuda_stream) if tune else None
        self.nout = self.R * Mx if offsets is None else Mx
        self.cdtype = torch.complex64 if code == lib.GT_C64 else torch.complex128
        self.version = 0

    def _set_nodes(self, x: torch.Tensor):
        if tuple(x.shape) != self.shape or x.dtype != self.xdtype:
            raise ValueError("the nodes must keep the shape and dtype given at construction")
        # (always: an optimiser may have changed the same tensor in place)
        self.plan.update_nodes(x.detach().contiguous())
        self.version += 1

    def __call__(self, fhat: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
        if fhat.dtype != self.cdtype:
            raise TypeError("fhat precision does not match the nodes")
        return _TrafoMoving.apply(fhat, x, self)

    def close(self):
        self.plan.close()


class _TrafoOnPlan(torch.autograd.Function):
    """f = F fhat on a prepared plan; backward gives the coefficients' gradient only."""

    @staticmethod
    def forward(ctx, fhat, owner):
        fhat_c = fhat.detach().contiguous()
        f = torch.empty(owner.nout, dtype=fhat.dtype, device=fhat.device)
        owner.plan.trafo(fhat_c, f)
        ctx.owner = owner
        ctx.shape_fhat = fhat.shape
        return f.view(owner.R, -1) if (owner.offsets is None and fhat.dim() == 2) else f

    @staticmethod
    def backward(ctx, gf):
        grad_fhat = None
        if ctx.needs_input_grad[0]:
            owner = ctx.owner
            grad_fhat = torch.empty(ctx.shape_fhat, dtype=gf.dtype, device=gf.device)
            owner.plan.adjoint(gf.contiguous(), grad_fhat)
        return grad_fhat, None


class GroupedTrafoFixedNodes:
    """Differentiable f = F(X) fhat for nodes fixed at construction: the plan (node copy and
    sort, the costly part of a call) is built once and reused by every call, which suits
    fitting coefficients to fixed data.  Gradients flow to fhat only; the nodes are copied
    when the object is built, so later changes to x are not seen (build a new object).

    x: (Mtot, d) real CUDA tensor; calls take fhat (R, |I|) or (|I|,) complex of the matching
    precision and return f as grouped_trafo does.  tune=True times the plan's launch forms
    once (gt_plan_tune, on the current stream)."""

    def __init__(self, x: torch.Tensor, d: int, ds: int, N: Sequence[int], R: int = 1,
                 offsets: Optional[Sequence[int]] = None, m: int = 0, sigma: float = 0.0, tune: bool = False):
        if not x.is_cuda:
            raise RuntimeError("grouped transform runs on the GPU only")
        code = lib.GT_C64 if x.dtype == torch.float32 else lib.GT_C128 if x.dtype == torch.float64 else None
        if code is None:
            raise TypeError("x must be float32 or float64")
        self.offsets = None if offsets is None else tuple(int(v) for v in offsets)
        self.R = int(R) if offsets is None else len(self.offsets) - 1
        x_c = x.detach().contiguous()
        Mx = x_c.shape[0]
        prob, keep = lib.make_problem(d, ds, N, M=Mx if offsets is None else 0, R=self.R, dtype=code, m=m,
                                      sigma=sigma, offsets=self.offsets)
        self.plan = lib.Plan(prob, x_c, keepalive=keep)
        self.tuning = self.plan.tune(torch.cuda.current_stream().cuda_stream) if tune else None
        self.nout = self.R * Mx if offsets is None else Mx
        self.cdtype = torch.complex64 if code == lib.GT_C64 else torch.complex128

    def __call__(self, fhat: torch.Tensor) -> torch.Tensor:
        if fhat.dtype != self.cdtype:
            raise TypeError("fhat precision does not match the nodes")
        return _TrafoOnPlan.apply(fhat, self)

    def close(self):
        self.plan.close()
