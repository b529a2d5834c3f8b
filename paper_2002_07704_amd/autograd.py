"""LNV band energy as a differentiable function of the block values of L, S, H.

E = 2 Tr[KH] with K = 3LSL - 2LSLSL (Sec. II.C.2, Eq. 4).  The forward pass
is lnv_eval (which also yields dE/dL = G); the backward pass returns G and,
when they are wanted, dE/dS and dE/dH from lnv_adjoint.  The adjoint keeps
nothing from the forward pass but G: the products L.S, L.S.L and H.L are
formed again in the backward pass, so the memory held between the two passes
is one vector on L's pattern.

Gradients are with respect to each stored entry (L, S and H are stored in
both triangles).  The inputs must be symmetric, as for lnv_eval; a symmetric
perturbation of the pair (i,j), (j,i) then changes E by G_ij + G_ji to first
order.
"""
from __future__ import annotations

import torch


def _check(t, name, nnzb, dev):
    if t.dtype != torch.float64 or t.device != dev or tuple(t.shape) != (nnzb, 4, 4):
        raise ValueError(f"{name}: expected float64 [{nnzb}, 4, 4] on {dev}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")


class LNVEnergy(torch.autograd.Function):
    """E = LNVEnergy.apply(L, S, H, system): values [nnzb, 4, 4] float64 on the
    patterns of ``system`` (an LNVSystem).  Uses the system's evaluation and
    adjoint workspaces on the current stream."""

    @staticmethod
    def forward(ctx, Lv, Sv, Hv, system):
        dev = Lv.device
        if dev.type != "cuda":
            raise ValueError("LNVEnergy: values must be on the GPU")
        _check(Lv, "L", system.pL.nnzb, dev)
        _check(Sv, "S", system.pS.nnzb, dev)
        _check(Hv, "H", system.pH.nnzb, dev)
        G = torch.empty_like(Lv)
        F = torch.empty_like(Lv)
        EN = torch.empty(2, dtype=torch.float64, device=Lv.device)
        system.eval_values(Lv, Sv, Hv, G, F, EN)
        ctx.system = system
        ctx.save_for_backward(Lv, Sv, Hv, G)
        return EN[0].clone()

    @staticmethod
    def backward(ctx, gE):
        Lv, Sv, Hv, G = ctx.saved_tensors
        system = ctx.system
        want_L, want_S, want_H = ctx.needs_input_grad[:3]
        dL = G * gE if want_L else None
        dS = dH = None
        if want_S or want_H:
            dS = torch.empty_like(Sv) if want_S else None
            dH = torch.empty_like(Hv) if want_H else None
            system.adjoint(Lv, Sv, Hv, dS=dS, dH=dH)
            dS = dS * gE if want_S else None
            dH = dH * gE if want_H else None
        return dL, dS, dH, None
