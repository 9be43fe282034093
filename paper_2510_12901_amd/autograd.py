"""torch.autograd.Function around the render: forward = project, bin_and_sort, composite;
backward = ut_composite_backward (hand-written adjoint replaying the saved tile lists)."""
from __future__ import annotations

import torch

from .render import (GaussianSet, Sensor, UT_ABK, actor_poses, actor_transform, actor_transform_backward, backward,
                     render, render_params)


class UTRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean, quat, log_scale, opacity_logit, feat, sh_degree: int, feat_kind: int,
                sensor: Sensor, abk=UT_ABK, params=None):
        g = GaussianSet(mean.detach().contiguous(), quat.detach().contiguous(), log_scale.detach().contiguous(),
                        opacity_logit.detach().contiguous(), feat.detach().contiguous(), sh_degree, feat_kind)
        prm = params or render_params()
        p, bins, out = render(g, sensor, abk, prm, state=True)
        ctx.state = (g, p, bins, out, sensor, prm)
        drop = out.drop if out.drop is not None else torch.zeros(0, device=mean.device)
        return out.feat, out.depth, out.alpha, drop

    @staticmethod
    def backward(ctx, g_feat, g_depth, g_alpha, g_drop):
        g, p, lists, out, sensor, prm = ctx.state
        if g_drop is not None and g_drop.numel() == 0:
            g_drop = None
        gr = backward(g, p, lists, sensor, out, g_feat, g_depth, g_alpha, g_drop, params=prm)
        return gr["mean"], gr["quat"], gr["log_scale"], gr["opacity_logit"], gr["feat"], None, None, None, None, None


def render_differentiable(g: GaussianSet, sensor: Sensor, abk=UT_ABK, params=None):
    """Differentiable render of a particle set whose tensors may require grad.
    Returns (feat [3,R], depth [R], alpha [R], drop [R] or empty)."""
    return UTRender.apply(g.mean, g.quat, g.log_scale, g.opacity_logit, g.feat, g.sh_degree, g.feat_kind,
                          sensor, abk, params)


class ActorTransform(torch.autograd.Function):
    """Object-frame (mean, quat) and actor poses [n_actors, 7] -> world-frame (mean, quat);
    the adjoint runs ut_actor_transform_backward (pose gradients included)."""
    @staticmethod
    def forward(ctx, mean, quat, poses, actor):
        g = GaussianSet(mean.detach().contiguous(), quat.detach().contiguous(), mean.new_empty(0), mean.new_empty(0),
                        mean.new_empty(0), 0, 0)
        pz = actor_poses(poses.detach()).to(mean.device)
        w = actor_transform(g, actor, pz)
        ctx.state = (g, actor, pz)
        return w.mean, w.quat

    @staticmethod
    def backward(ctx, g_mean, g_quat):
        g, actor, pz = ctx.state
        g_mean = torch.zeros_like(g.mean) if g_mean is None else g_mean
        g_quat = torch.zeros_like(g.quat) if g_quat is None else g_quat
        dm, dq, dp = actor_transform_backward(g, actor, pz, g_mean, g_quat, pose_grad=ctx.needs_input_grad[2])
        return dm, dq, (dp.float() if dp is not None else None), None


def transform_differentiable(g: GaussianSet, actor: torch.Tensor, poses: torch.Tensor) -> GaussianSet:
    """World-frame particle set whose mean and quaternion carry gradients back to the
    object-frame parameters and to the poses (a float32 [n_actors, 7] tensor)."""
    mean_w, quat_w = ActorTransform.apply(g.mean, g.quat, poses, actor)
    return g.with_params(mean_w, quat_w, g.log_scale, g.opacity_logit, g.feat)

