"""torch.autograd.Function over the library's reverse-mode entry point.

H(w_+, w_-; L) of Eq. (3) is holomorphic in the fields, so for a complex
output gradient g the field gradients are g * conj(dH/dw) (PyTorch's
convention for holomorphic maps).  The box edges L = (L_x, L_y, L_z) are a
real input: their gradient is Re(g * conj(dH/dL)), with dH/dL the box
derivative at fixed grid values of the fields (each edge varied alone).
When any input requires a gradient, the forward pass runs pft_adjoint once,
which yields H, dH/dw and dH/dL together; the backward pass only scales the
stored derivatives.
"""
from __future__ import annotations

import torch

from . import binding


def _sync_box(pft: "binding.Context", L: torch.Tensor | None):
    """Move the context to the box edges L (a 3-element real tensor) if they
    differ from its current ones."""
    if L is None:
        return
    if L.shape != (3,) or L.dtype != torch.float64:
        raise ValueError("L must be a float64 tensor of shape (3,)")
    lx, ly, lz = (float(v) for v in L.detach().cpu())
    p = pft.params
    if (lx, ly, lz) != (p.lx, p.ly, p.lz):
        pft.pft_set_box(lx, ly, lz)


class PftHamiltonian(torch.autograd.Function):
    @staticmethod
    def forward(fctx, pft: "binding.Context", w_plus: torch.Tensor, w_minus: torch.Tensor,
                L: torch.Tensor | None = None, ckpt_every: int = 0):
        _sync_box(pft, L)
        H = torch.empty(1, dtype=torch.complex128, device=w_plus.device)
        need_L = L is not None and L.requires_grad
        if w_plus.requires_grad or w_minus.requires_grad or need_L:
            gp = torch.empty_like(w_plus)
            gm = torch.empty_like(w_minus)
            dL = torch.empty(3, dtype=torch.complex128, device=w_plus.device) if need_L else None
            pft.pft_adjoint(w_plus.detach(), w_minus.detach(), gp, gm, dL, H, ckpt_every)
            fctx.save_for_backward(gp, gm, dL)
            fctx.L_device = L.device if L is not None else None
        else:
            pft.pft_propagate(w_plus, w_minus)
            pft.pft_hamiltonian(w_plus, w_minus, H)
        return H[0]

    @staticmethod
    def backward(fctx, g):
        gp, gm, dL = fctx.saved_tensors
        gL = None if dL is None else (g * dL.conj()).real.to(device=fctx.L_device, dtype=torch.float64)
        return None, g * gp.conj(), g * gm.conj(), gL, None


def hamiltonian(pft: "binding.Context", w_plus: torch.Tensor, w_minus: torch.Tensor,
                L: torch.Tensor | None = None, ckpt_every: int = 0):
    """H[w_+, w_-] as a differentiable 0-dim complex128 tensor.  L, if given,
    is a float64 tensor (device or host) of the box edges in R_g: the context
    is moved to that box first (pft_set_box), and L is differentiable."""
    return PftHamiltonian.apply(pft, w_plus, w_minus, L, ckpt_every)
