"""torch.autograd.Function over the element-wise injections and their adjoint.

Forward calls ``pf_injections_elementwise``; backward calls the hand-written
adjoint kernel ``pf_injections_vjp`` (the gradient of
sum_i lam_P,i P_i + lam_Q,i Q_i with respect to vm and va, J never formed).
Both run on torch's current stream.  Double backward is not supported.
"""
from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable

from . import pf


class Injections(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid: "pf.Grid", vm: torch.Tensor, va: torch.Tensor):
        vm = vm.contiguous()
        va = va.contiguous()
        p = torch.empty_like(vm)
        q = torch.empty_like(vm)
        pf.pf_injections_elementwise(grid, vm, va, p, q)
        ctx.grid = grid
        ctx.save_for_backward(vm, va)
        return p, q

    @staticmethod
    @once_differentiable
    def backward(ctx, gp: torch.Tensor, gq: torch.Tensor):
        vm, va = ctx.saved_tensors
        gp = torch.zeros_like(vm) if gp is None else gp.contiguous()
        gq = torch.zeros_like(vm) if gq is None else gq.contiguous()
        g_vm = torch.empty_like(vm)
        g_va = torch.empty_like(vm)
        pf.pf_injections_vjp(ctx.grid, vm, va, gp, gq, g_vm, g_va)
        return None, g_vm, g_va


def injections(grid: "pf.Grid", vm: torch.Tensor, va: torch.Tensor):
    """(P, Q) = S(vm, va) by the element-wise method, differentiable in vm and va."""
    return Injections.apply(grid, vm, va)
