"""torch.autograd.Function over the HIP rollout: costs forward, the
hand-written adjoint kernel backward (argument marshalling only)."""
from __future__ import annotations

import torch

from . import plan as P


class RolloutCost(torch.autograd.Function):
    """J = RolloutCost.apply(controls, planner, state0, checkpoint_every).

    controls: [N][2][K] float32 CUDA tensor (raw controls, clamped inside);
    planner:  a plan.Planner with its terrain set; returns J [K]. The backward
    pass recomputes the rollout from checkpoints every `checkpoint_every`
    control intervals and returns dL/dcontrols = sum_k (dL/dJ_k) dJ_k/du."""

    @staticmethod
    def forward(ctx, controls, planner, state0, checkpoint_every=10):
        controls = controls.contiguous()
        K = controls.shape[2]
        J = torch.empty(K, device=controls.device, dtype=torch.float32)
        planner.rollout(state0, controls, J)
        ctx.save_for_backward(controls)
        ctx.planner = planner
        ctx.state0 = state0
        ctx.ckpt = int(checkpoint_every)
        return J

    @staticmethod
    def backward(ctx, gJ):
        (controls,) = ctx.saved_tensors
        K = controls.shape[2]
        cost = torch.empty(K, device=controls.device, dtype=torch.float32)
        grad = torch.empty_like(controls)
        P.plan_rollout_grad(ctx.planner.ctx, ctx.state0, controls, cost, grad,
                            weight=gJ.contiguous().float(), checkpoint_every=ctx.ckpt)
        return grad, None, None, None
