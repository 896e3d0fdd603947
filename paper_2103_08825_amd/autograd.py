"""torch.autograd.Function over the sweep and its hand-written adjoint.

    u_T = StencilFn.apply(u0, coeffs, shape_spec, T, ckpt)

differentiates u_T with respect to the initial field u0 and the weights
coeffs (canonical order).  The forward pass is stencil_run; the backward pass
is stencil_adjoint (mirrored stencil run backwards in time, checkpoints every
`ckpt` steps, FP64 coefficient sums).  Plans are cached per weight values.
"""
from __future__ import annotations

import torch

from .api import Plan


class StencilSpec:
    """Everything of a plan except its weights."""

    def __init__(self, shape, r: int, kind: int, bc: int, dtype, method: str = "auto"):
        self.shape = tuple(int(s) for s in shape)
        self.r, self.kind, self.bc, self.dtype, self.method = int(r), int(kind), int(bc), dtype, method
        self._cache = {}

    def plan(self, coeffs: torch.Tensor) -> Plan:
        key = tuple(float(c) for c in coeffs.detach().to("cpu", torch.float64).tolist())
        p = self._cache.get(key)
        if p is None:
            if len(self._cache) > 8:
                self._cache.clear()
            p = Plan(self.shape, self.r, self.kind, list(key), self.bc, self.dtype, method=self.method)
            self._cache[key] = p
        return p


class StencilFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0: torch.Tensor, coeffs: torch.Tensor, spec: StencilSpec, T: int, ckpt: int = 10):
        plan = spec.plan(coeffs)
        u0c = u0.contiguous()
        ctx.save_for_backward(u0c, coeffs)
        ctx.plan, ctx.T, ctx.ckpt = plan, int(T), int(ckpt)
        return plan.run(u0c, int(T))

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        u0, coeffs = ctx.saved_tensors
        grad_u0, grad_c = ctx.plan.adjoint(u0, g.contiguous().to(u0.dtype), ctx.T, ctx.ckpt)
        gu = grad_u0 if ctx.needs_input_grad[0] else None
        gc = grad_c.to(coeffs.dtype).to(coeffs.device) if ctx.needs_input_grad[1] else None
        return gu, gc, None, None, None
