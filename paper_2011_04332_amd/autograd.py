"""torch.autograd.Function over the differentiable rollout.

Forward: set the per-cell weights, load the initial state, run n_steps
projective-dynamics steps with checkpoints (npfem_rollout). Backward: the
hand-written adjoint in the HIP library (npfem_rollout_adjoint) returns the
gradients with respect to the per-cell weights (stretch, area, bend, volume),
the constant external forces and the initial state.
"""
from __future__ import annotations

import torch


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, weights, forces, x0, v0, batch, dt, n_iter, n_steps, ckpt_every):
        batch.set_weights(weights.detach().to("cpu", torch.float64).numpy())
        with torch.no_grad():
            batch.pos.copy_(x0)
            batch.vel.copy_(v0)
        f = forces.detach().contiguous()
        batch.rollout(f, dt, n_iter, n_steps, ckpt_every)
        ctx.batch = batch
        ctx.keep = f  # the rollout recorded this buffer's address
        ctx.wdev = weights.device
        return batch.pos.clone(), batch.vel.clone()

    @staticmethod
    def backward(ctx, gx, gv):
        b = ctx.batch
        gx = torch.zeros_like(b.pos) if gx is None else gx.contiguous()
        gv = None if gv is None else gv.contiguous()
        dw, df, dx0, dv0 = b.rollout_adjoint(gx, gv)
        return dw.to(ctx.wdev), df, dx0, dv0, None, None, None, None, None


def rollout(batch, weights, forces, x0, v0, dt, n_iter, n_steps, ckpt_every=10):
    """Differentiable (x_T, v_T) of a batch rollout."""
    return Rollout.apply(weights, forces, x0, v0, batch, dt, n_iter, n_steps, ckpt_every)
