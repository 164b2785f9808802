"""F_V as a differentiable torch function (eq. 2.4): the forward pass is
the library's energy kernel, the backward pass its hand-written gradient
kernel (Section 3.4), with the upstream gradient folded into the kernel's
quadrature weights (tmop_gradient_scaled)."""
from __future__ import annotations

import torch

from .tmop import Context


class TMOPEnergy(torch.autograd.Function):
    """F = TMOPEnergy.apply(x, ctx) for x of shape (dim, n_node), float64 on
    the context's device.  Returns a 0-dim float64 tensor on that device."""

    @staticmethod
    def forward(fctx, x: torch.Tensor, tctx: Context):
        F, _, _ = tctx.energy(x.contiguous())
        fctx.tctx = tctx
        fctx.save_for_backward(x)
        return torch.tensor(F, dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(fctx, grad_out: torch.Tensor):
        (x,) = fctx.saved_tensors
        scale = grad_out.detach().to(dtype=torch.float64).reshape(1)
        g = fctx.tctx.gradient_scaled(x.detach().contiguous(), scale)
        return g, None


def tmop_energy_fn(x: torch.Tensor, tctx: Context) -> torch.Tensor:
    return TMOPEnergy.apply(x, tctx)
