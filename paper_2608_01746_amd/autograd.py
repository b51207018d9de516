"""torch.autograd binding of the far-field loss (the adjoint of Eqs. 2-3).

PtychoLoss.apply(O, P, I, pos, kind, eps, batch) returns the float64 loss
summed over positions and detector pixels; backward calls the library's
adjoint kernels, which recompute the exit waves chunk by chunk instead of
storing them.  Gradients follow PyTorch's complex convention
(dL/dRe + i dL/dIm), so they are returned unchanged."""
from __future__ import annotations

import torch

from . import api


class PtychoLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, O, P, I, pos, kind="poisson", eps=1e-6, batch=32):
        loss, _, _ = api.ptycho_grad(O.detach(), P.detach(), I, pos, kind, eps, batch, None,
                                     need_gO=False, need_gP=False)
        ctx.save_for_backward(O, P, I)
        ctx.pos, ctx.kind, ctx.eps, ctx.batch = pos, kind, eps, batch
        return loss

    @staticmethod
    def backward(ctx, g):
        O, P, I = ctx.saved_tensors
        need_O, need_P = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_O or need_P):
            return (None,) * 7
        # the upstream factor stays on the device: the kernels read it in place
        up = g.detach().to(device=O.device, dtype=torch.float64).reshape(())
        _, gO, gP = api.ptycho_grad(O.detach(), P.detach(), I, ctx.pos, ctx.kind, ctx.eps, ctx.batch, up,
                                    need_gO=need_O, need_gP=need_P)
        return gO, gP, None, None, None, None, None


def ptycho_loss(O, P, I, pos, kind="poisson", eps=1e-6, batch=32):
    return PtychoLoss.apply(O, P, I, pos, kind, eps, batch)
