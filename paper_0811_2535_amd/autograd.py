"""Differentiable transform: ``torch.autograd.Function`` whose backward is the
adjoint transform.

For y = F_s x with (F_s)[k, j] = exp(s 2 pi i j k / n), the adjoint is
F_s^H = F_{-s} (unnormalized).  PyTorch propagates the conjugate Wirtinger
gradient, so for a real loss L the gradient with respect to x is
F_s^H (dL/dy) = F_{-s}(dL/dy): the backward runs the same kernels with the
opposite sign and saves nothing from the forward.
"""
from __future__ import annotations

import torch

from .binding import fft


class LiftFFT(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, sign: int = -1) -> torch.Tensor:
        ctx.sign = int(sign)
        return fft(x, ctx.sign)

    @staticmethod
    def backward(ctx, grad_y: torch.Tensor):
        return fft(grad_y.contiguous(), -ctx.sign), None


def fft_autograd(x: torch.Tensor, sign: int = -1) -> torch.Tensor:
    return LiftFFT.apply(x, sign)
