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
        # a private copy: the library records the forces buffer's address for
        # the backward pass, so later in-place changes of the caller's tensor
        # must not reach it
        f = forces.detach().clone().contiguous()
        batch.rollout(f, dt, n_iter, n_steps, ckpt_every)
        ctx.batch = batch
        ctx.keep = f
        ctx.generation = batch.rollout_generation
        ctx.wdev = weights.device
        return batch.pos.clone(), batch.vel.clone()

    @staticmethod
    def backward(ctx, gx, gv):
        b = ctx.batch
        if b.rollout_generation != ctx.generation:
            raise RuntimeError("the batch ran another rollout after this one: its checkpoints "
                               "are gone (one Rollout.apply per batch between backward passes)")
        gx = torch.zeros_like(b.pos) if gx is None else gx.contiguous()
        gv = None if gv is None else gv.contiguous()
        dw, df, dx0, dv0 = b.rollout_adjoint(gx, gv)
        return dw.to(ctx.wdev), df, dx0, dv0, None, None, None, None, None


def rollout(batch, weights, forces, x0, v0, dt, n_iter, n_steps, ckpt_every=10):
    """Differentiable (x_T, v_T) of a batch rollout."""
    return Rollout.apply(weights, forces, x0, v0, batch, dt, n_iter, n_steps, ckpt_every)
