"""Differentiable exchange energy: E_x behind a torch.autograd.Function.

Forward calls fock_energy; backward calls fock_energy_backward, which
recomputes the pair densities instead of storing them.  PyTorch's gradient of
a real loss with respect to a complex tensor z is 2 dL/d(conj z) (the
conjugate Wirtinger derivative, doubled); the C ABI returns dE/d(conj z), so
the backward passes 2 * grad_out as the scale.  When the occupied and target
blocks are the same tensor, autograd adds the two contributions.
"""
from __future__ import annotations

import torch

from . import fock


class ExchangeEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c_occ, c_tgt, f_occ, g_tgt, cell, q):
        ws = fock.workspace(cell, fock.dtype_code(c_occ), c_occ.shape[0], c_tgt.shape[0], c_occ.device)
        ex = fock.fock_energy(cell, q, c_occ, f_occ, c_tgt, g_tgt, ws=ws)
        ctx.save_for_backward(c_occ, c_tgt, f_occ, g_tgt)
        ctx.cell, ctx.q = cell, q
        return ex

    @staticmethod
    def backward(ctx, grad):
        c_occ, c_tgt, f_occ, g_tgt = ctx.saved_tensors
        scale = grad.detach().to(device=c_occ.device, dtype=torch.float64).mul(2.0).contiguous()
        need_o, need_t = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        go = torch.empty_like(c_occ) if need_o else None
        gt = torch.empty_like(c_tgt) if need_t else None
        if need_o or need_t:
            ws = fock.workspace(ctx.cell, fock.dtype_code(c_occ), c_occ.shape[0], c_tgt.shape[0], c_occ.device)
            fock.fock_energy_backward(ctx.cell, ctx.q, c_occ, f_occ, c_tgt, g_tgt, scale, go, gt, ws=ws)
        return go, gt, None, None, None, None


def exchange_energy(c_occ, c_tgt, f_occ, g_tgt, cell, q=(0.0, 0.0, 0.0)):
    return ExchangeEnergy.apply(c_occ, c_tgt, f_occ, g_tgt, cell, q)


class ExchangeEnergyKMesh(torch.autograd.Function):
    """E_x over a k-point mesh for C [nk, nb, npw]; W [nk, nb] are occupation / N_k."""

    @staticmethod
    def forward(ctx, C, W, cell, kpts):
        ws = fock.workspace_kmesh(cell, fock.dtype_code(C), C.shape[0], C.shape[1], C.device)
        ex = fock.fock_energy_kmesh(cell, kpts, C, W, ws=ws)
        ctx.save_for_backward(C, W)
        ctx.cell, ctx.kpts = cell, kpts
        return ex

    @staticmethod
    def backward(ctx, grad):
        C, W = ctx.saved_tensors
        if not ctx.needs_input_grad[0]:
            return None, None, None, None
        scale = grad.detach().to(device=C.device, dtype=torch.float64).mul(2.0).contiguous()
        G = torch.empty_like(C)
        ws = fock.workspace_kmesh(ctx.cell, fock.dtype_code(C), C.shape[0], C.shape[1], C.device)
        fock.fock_energy_kmesh_backward(ctx.cell, ctx.kpts, C, W, scale, [G[k] for k in range(C.shape[0])], ws=ws)
        return G, None, None, None


def exchange_energy_kmesh(C, W, cell, kpts):
    return ExchangeEnergyKMesh.apply(C, W, cell, kpts)
