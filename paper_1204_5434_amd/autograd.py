"""torch.autograd.Function over the library's reverse-mode entry point.

H(w_+, w_-) of Eq. (3) is holomorphic in the fields, so for a complex
output gradient g the input gradients are g * conj(dH/dw) (PyTorch's
convention for holomorphic maps).  When any input requires a gradient, the
forward pass runs pft_adjoint once, which yields H and dH/dw together; the
backward pass only scales the stored derivatives.
"""
from __future__ import annotations

import torch

from . import binding


class PftHamiltonian(torch.autograd.Function):
    @staticmethod
    def forward(fctx, pft: "binding.Context", w_plus: torch.Tensor, w_minus: torch.Tensor,
                ckpt_every: int = 0):
        H = torch.empty(1, dtype=torch.complex128, device=w_plus.device)
        if w_plus.requires_grad or w_minus.requires_grad:
            gp = torch.empty_like(w_plus)
            gm = torch.empty_like(w_minus)
            pft.pft_adjoint(w_plus.detach(), w_minus.detach(), gp, gm, None, H, ckpt_every)
            fctx.save_for_backward(gp, gm)
        else:
            pft.pft_propagate(w_plus, w_minus)
            pft.pft_hamiltonian(w_plus, w_minus, H)
        return H[0]

    @staticmethod
    def backward(fctx, g):
        gp, gm = fctx.saved_tensors
        return None, g * gp.conj(), g * gm.conj(), None


def hamiltonian(pft: "binding.Context", w_plus: torch.Tensor, w_minus: torch.Tensor, ckpt_every: int = 0):
    """H[w_+, w_-] as a differentiable 0-dim complex128 tensor."""
    return PftHamiltonian.apply(pft, w_plus, w_minus, ckpt_every)
