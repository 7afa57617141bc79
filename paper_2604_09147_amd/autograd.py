"""torch.autograd.Function over the H_h product: forward y = H^ x, backward
grad_x = H^^T grad_y (the transposed product: roles of U_b and V_b swapped,
dense diagonal blocks applied from transposed copies stored at build time).
Both directions run in the native library; torch only supplies tensors and the
stream."""
from __future__ import annotations

import torch

from .hh import HMatrix


class HHMatvec(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, hmat: HMatrix) -> torch.Tensor:
        ctx.hmat = hmat
        return hmat.matvec(x.detach())

    @staticmethod
    def backward(ctx, grad_y: torch.Tensor):
        return ctx.hmat.matvec_t(grad_y.contiguous()), None


def hh_apply(hmat: HMatrix, x: torch.Tensor) -> torch.Tensor:
    """Differentiable y = H^ x."""
    return HHMatvec.apply(x, hmat)
