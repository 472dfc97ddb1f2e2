"""torch.autograd.Function around the codec-fit loss and its hand-written
gradient (hc_codec_step without the optimizer step).

The forward pass runs the loss kernels, which produce dL/dWt_E and dL/dWt_D
in the same launch; backward scales those by the incoming gradient.  The
data batches are constants of the loss: no gradient flows to them.
"""

from __future__ import annotations

import torch

from . import ops


class CodecLoss(torch.autograd.Function):
    """L = (1/N) sum_i |D E a_i - a_i|^2 + |D E b_i - b_i|^2
             + lam |D (E a_i (.) E b_i) - a_i * b_i|^2,
    E = softplus_beta(Wt_E), D = softplus_beta(Wt_D)."""

    @staticmethod
    def forward(ctx, wt_e, wt_d, a, b, lam: float = 1.0, beta: float = 10.0):
        if a.requires_grad or b.requires_grad:
            raise ValueError("CodecLoss differentiates with respect to the codec parameters only")
        we, wd = wt_e.detach().contiguous(), wt_d.detach().contiguous()
        a, b = a.detach().contiguous(), b.detach().contiguous()
        ge, gd = torch.empty_like(we), torch.empty_like(wd)
        loss = ops.codec_step(we, wd, a, b, a.shape[0], lam=lam, beta=beta, grad_e=ge, grad_d=gd)
        ctx.save_for_backward(ge, gd)
        return loss

    @staticmethod
    def backward(ctx, grad_out):
        ge, gd = ctx.saved_tensors
        return grad_out * ge, grad_out * gd, None, None, None, None


def codec_loss(wt_e, wt_d, a, b, lam: float = 1.0, beta: float = 10.0):
    return CodecLoss.apply(wt_e, wt_d, a, b, lam, beta)
