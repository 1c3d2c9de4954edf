"""Autograd through the emulated product: a torch.autograd.Function whose
forward keeps the residue planes of X' and W' and whose backward forms
dX = dY W^T and dW = X^T dY through the same emulation, reusing them
(ozemu_dgemm_fwd_cache / ozemu_dgemm_bwd). Marshalling only: every step
runs in libozemu's kernels.

    from paper_2609_37693_amd import Plan
    from paper_2609_37693_amd.autograd import emulated_matmul
    Y = emulated_matmul(X, W, Plan(16, "W"))   # float64 CUDA tensors
"""
from __future__ import annotations

import torch

from . import Plan, dgemm_bwd, dgemm_fwd_cache

__all__ = ["EmulatedMatmul", "emulated_matmul", "EmulatedLinear"]


class EmulatedMatmul(torch.autograd.Function):
    """Y = X @ W (X m x k, W k x n, float64 on a HIP device)."""

    @staticmethod
    def forward(ctx, X, W, plan):
        Y, cache = dgemm_fwd_cache(X.detach(), W.detach(), plan)
        ctx.cache = cache
        return Y

    @staticmethod
    def backward(ctx, dY):
        cache = ctx.cache
        need_dx, need_dw = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        # the cache stays on ctx (freed with the graph), so a graph kept with
        # retain_graph=True can run its backward again
        dX, dW = dgemm_bwd(dY.contiguous(), cache, need_dx=need_dx, need_dw=need_dw)
        return dX, dW, None


def emulated_matmul(X, W, plan: Plan):
    return EmulatedMatmul.apply(X, W, plan)


class EmulatedLinear(torch.nn.Module):
    """y = x W with W (in_features x out_features), no bias, through the
    emulated product in both directions."""

    def __init__(self, weight: torch.Tensor, plan: Plan):
        super().__init__()
        self.weight = torch.nn.Parameter(weight)
        self.plan = plan

    def forward(self, x):
        return emulated_matmul(x, self.weight, self.plan)
