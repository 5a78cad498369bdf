"""torch.autograd.Function front ends of the adjoint rollout kernel.

``MeanReturn.apply(actions, model, s0, H, gamma, goal, particles, seed)`` is
the mean discounted return of rollouts driven by continuous action sequences;
its backward hands the gradient computed by the adjoint kernel (the forward
launch runs the checkpointed forward and the reverse sweep together) to
autograd.  ``DistillLoss.apply(*flat_weights, desc, s0, actions, targets, H,
seed)`` is the rollout distillation loss as a function of the transition
network's weights; each call packs the given weights into a device model.
"""
from __future__ import annotations

import copy

import torch

from . import Model, VOILA_OBJ_DISTILL, VOILA_OBJ_RETURN, rollout_grad, unflatten_params


class MeanReturn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, actions, model, s0, H, gamma, goal, particles, seed, checkpoint=5):
        loss, _, ga = rollout_grad(model, s0, actions.detach().contiguous(), H, VOILA_OBJ_RETURN, gamma=gamma,
                                   goal=goal, particles=particles, seed=seed, checkpoint=checkpoint,
                                   want_params=False, want_actions=True)
        ctx.save_for_backward(ga)
        return loss[0]

    @staticmethod
    def backward(ctx, grad_out):
        (ga,) = ctx.saved_tensors
        return (grad_out * ga,) + (None,) * 8


class DistillLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, *args):
        *flat, desc, s0, actions, targets, H, seed = args
        layers = [(flat[2 * j].detach().cpu().numpy(), flat[2 * j + 1].detach().cpu().numpy())
                  for j in range(len(flat) // 2)]
        d = copy.copy(desc)
        d.trans = layers
        m = Model(d, compute="f32", device=s0.device.index or 0)
        loss, gp, _ = rollout_grad(m, s0, actions, H, VOILA_OBJ_DISTILL, targets=targets, seed=seed)
        grads = [t for pair in unflatten_params(m, gp) for t in pair]
        ctx.grads = [g.to(f.device).reshape(f.shape) for g, f in zip(grads, flat)]
        m.close()
        return loss[0]

    @staticmethod
    def backward(ctx, grad_out):
        return tuple(grad_out.to(g.device) * g for g in ctx.grads) + (None,) * 6
