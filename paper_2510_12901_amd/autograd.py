"""torch.autograd.Function around the render: forward = project, bin_and_sort, composite;
backward = ut_composite_backward (hand-written adjoint replaying the saved tile lists)."""
from __future__ import annotations

import torch

from .render import (GaussianSet, RenderOut, Sensor, UT_ABK, actor_poses, actor_transform, actor_transform_backward, backward,
                     render, render_params)


class UTRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean, quat, log_scale, opacity_logit, feat, sh_degree: int, feat_kind: int,
                sensor: Sensor, abk=UT_ABK, params=None):
        g = GaussianSet(mean.detach().contiguous(), quat.detach().contiguous(), log_scale.detach().contiguous(),
                        opacity_logit.detach().contiguous(), feat.detach().contiguous(), sh_degree, feat_kind)
        prm = params or render_params()
        p, bins, out = render(g, sensor, abk, prm, state=True)
        drop = out.drop if out.drop is not None else torch.zeros(0, device=mean.device)
        # the returned tensors go through save_for_backward (no output -> ctx -> output cycle,
        # and autograd refuses a backward after an in-place edit of them: the adjoint reads
        # feat for the ray-drop derivative); only the adjoint state that is not returned stays
        # on ctx
        ctx.save_for_backward(out.feat, out.depth, out.alpha, drop)
        ctx.state = (g, p, bins, out.t_final, out.n_proc, out.tile_end, sensor, prm)
        return out.feat, out.depth, out.alpha, drop

    @staticmethod
    def backward(ctx, g_feat, g_depth, g_alpha, g_drop):
        g, p, lists, t_final, n_proc, tile_end, sensor, prm = ctx.state
        feat, depth, alpha, drop = ctx.saved_tensors
        out = RenderOut(feat, depth, alpha, drop if drop.numel() else None, t_final, n_proc, tile_end=tile_end)
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

