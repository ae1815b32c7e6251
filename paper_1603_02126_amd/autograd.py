"""Differentiable fixed-gain imaging: gains -> time-averaged EPIC image.

`epic_image(gains, plan, array, efield, n_samples)` returns the image
[F, ny, nx] of epic_image and, under autograd, back-propagates through the
library's hand-written adjoint (epic_image_adjoint), which recomputes every
per-sample transform instead of storing it.  Gradients follow PyTorch's
convention for complex leaves: dL/dRe g + i dL/dIm g.
"""
from __future__ import annotations

import torch


class EpicImageFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gains, plan, array, efield, n_samples):
        g = gains.detach().to(torch.complex128).contiguous()
        image = plan.image(array, efield, n_samples, g)
        ctx.plan, ctx.array, ctx.efield, ctx.n_samples = plan, array, efield, n_samples
        ctx.in_dtype = gains.dtype
        ctx.save_for_backward(g)
        return image

    @staticmethod
    def backward(ctx, dL_dI):
        (g,) = ctx.saved_tensors
        grad = ctx.plan.image_adjoint(ctx.array, ctx.efield, ctx.n_samples, g,
                                      dL_dI.detach().to(torch.float32).contiguous())
        return grad.to(ctx.in_dtype), None, None, None, None


def epic_image(gains: torch.Tensor, plan, array: int, efield: torch.Tensor, n_samples: int) -> torch.Tensor:
    """Time-averaged image of `array` with fixed gains [F, Na] (complex)."""
    return EpicImageFn.apply(gains, plan, array, efield, n_samples)
