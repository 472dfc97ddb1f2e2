"""torch.autograd.Functions around the codec-fit losses (the two-term squared
error and the four-term loss of Eq. 8) and their hand-written gradients
(hc_codec_step without the optimizer step).

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
        return _forward(ctx, wt_e, wt_d, a, b, dict(lam=lam, beta=beta))

    @staticmethod
    def backward(ctx, grad_out):
        ge, gd = ctx.saved_tensors
        return grad_out * ge, grad_out * gd, None, None, None, None


class CodecLossEq8(torch.autograd.Function):
    """The four-term loss of Eq. 8,
    w_e2e L_e2e + w_rec L_rec + w_code L_code + w_col L_col,
    on E = softplus_beta(Wt_E), D = softplus_beta(Wt_D); T is the 3 x n
    colour-matching matrix (a constant of the loss)."""

    @staticmethod
    def forward(ctx, wt_e, wt_d, a, b, T, weights=ops.EQ8_WEIGHTS, beta: float = 10.0,
                cos_eps: float = 1e-8):
        if T.requires_grad:
            raise ValueError("CodecLossEq8 differentiates with respect to the codec parameters only")
        return _forward(ctx, wt_e, wt_d, a, b,
                        dict(beta=beta, objective="eq8", T=T.detach().contiguous(),
                             weights=weights, cos_eps=cos_eps))

    @staticmethod
    def backward(ctx, grad_out):
        ge, gd = ctx.saved_tensors
        return grad_out * ge, grad_out * gd, None, None, None, None, None, None


def _forward(ctx, wt_e, wt_d, a, b, kw):
    if a.requires_grad or b.requires_grad:
        raise ValueError("the codec losses differentiate with respect to the codec parameters only")
    we, wd = wt_e.detach().contiguous(), wt_d.detach().contiguous()
    a, b = a.detach().contiguous(), b.detach().contiguous()
    ge, gd = torch.empty_like(we), torch.empty_like(wd)
    loss = ops.codec_step(we, wd, a, b, a.shape[0], grad_e=ge, grad_d=gd, **kw)
    ctx.save_for_backward(ge, gd)
    return loss


def codec_loss(wt_e, wt_d, a, b, lam: float = 1.0, beta: float = 10.0):
    return CodecLoss.apply(wt_e, wt_d, a, b, lam, beta)


def codec_loss_eq8(wt_e, wt_d, a, b, T, weights=ops.EQ8_WEIGHTS, beta: float = 10.0,
                   cos_eps: float = 1e-8):
    return CodecLossEq8.apply(wt_e, wt_d, a, b, T, tuple(weights), beta, cos_eps)
