"""torch.autograd.Function over the HIP adjoint of one MD window.

The forward pass and the checkpointed reverse sweep both run in the library
(`mdlg_adjoint`): the forward call computes the loss and every gradient at
once, and backward only scales them by the incoming gradient.
"""
from __future__ import annotations

import torch


class WindowLoss(torch.autograd.Function):
    """L(v0, eps, sigma): the displacement loss of `window` velocity-Verlet
    steps from the system's current positions with initial velocities v0
    (device tensor, id order).  The system's positions and velocities are
    restored afterwards, so repeated calls evaluate the same window."""

    @staticmethod
    def forward(ctx, v0, eps, sigma, system, window, ckpt_every, loss):
        saved = system.get_state()
        system.set_potential(float(eps), float(sigma))
        L, ge, gs, gv = system.adjoint(window, ckpt_every, loss, v0=v0)
        system.set_state(saved["ucell"], saved["off"], saved["vel"], saved["prev_ucell"],
                         saved["prev_off"])
        ctx.save_for_backward(gv.to(v0.dtype))
        ctx.gp = (ge, gs)
        ctx.dtypes = (eps.dtype, sigma.dtype)
        return torch.tensor(L, dtype=torch.float64, device=v0.device)

    @staticmethod
    def backward(ctx, g):
        (gv,) = ctx.saved_tensors
        ge, gs = ctx.gp
        gd = g.detach()
        return (gd.to(gv.dtype) * gv, (gd * ge).to(ctx.dtypes[0]).reshape(()),
                (gd * gs).to(ctx.dtypes[1]).reshape(()), None, None, None, None)


def window_loss(system, v0, eps, sigma, window=20, ckpt_every=5, loss="msd"):
    """Differentiable displacement loss of one MD window (see WindowLoss)."""
    return WindowLoss.apply(v0, eps, sigma, system, window, ckpt_every, loss)
