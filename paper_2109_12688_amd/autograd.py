"""torch.autograd over the differentiated warping (argument marshalling only).

`one_warping_ssd(moving, lam, fixed, theta, order, iters, checkpoint)` is
L = sum (moving(x + w(x)) - fixed(x))^2 with w the velocity of one warping
(`iters` unrolled Nesterov-ADMM iterations from u = 0), differentiable with
respect to `moving` and `lam` (a 0-d tensor, best on the CPU: the library
takes lambda as a host value, so a GPU tensor costs a synchronisation).
When a gradient is required the forward pass calls the library's gradient
entry point, which runs the iterations with checkpoints every `checkpoint`
iterations and the reverse pass in its own kernels, and the backward pass
only scales the stored gradients by the incoming gradient; otherwise the
forward pass computes the loss alone (no reverse pass).
"""
from __future__ import annotations

import torch

from . import api


class _OneWarpingSSD(torch.autograd.Function):
    @staticmethod
    def forward(ctx, moving, lam, fixed, theta, order, iters, checkpoint):
        # lambda is a host parameter of the library: a CPU tensor costs nothing,
        # a GPU tensor one synchronisation
        lam_f = float(lam.item()) if isinstance(lam, torch.Tensor) else float(lam)
        need = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
        loss, dmov, dlam = api.ssd_grad(fixed.contiguous(), moving.contiguous(), lam_f, theta, order, iters,
                                        checkpoint, loss_only=not need)
        if need:
            ctx.save_for_backward(dmov, dlam)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        dmov, dlam = ctx.saved_tensors
        g = grad_loss.to(torch.float64)
        gm = (g * dmov.to(torch.float64)).to(dmov.dtype) if ctx.needs_input_grad[0] else None
        gl = (g * dlam).to(torch.float64) if ctx.needs_input_grad[1] else None
        return gm, gl, None, None, None, None, None


def one_warping_ssd(moving: torch.Tensor, lam: torch.Tensor, fixed: torch.Tensor, theta: float,
                    order: int, iters: int, checkpoint: int = 5) -> torch.Tensor:
    return _OneWarpingSSD.apply(moving, lam, fixed, theta, order, iters, checkpoint)
