"""Rigid actor transforms of the scene graph on the GPU (through the C-ABI) against the FP64
oracle: the transform itself, a render of a scene with actors, the adjoint (object-frame
parameters and poses) and the end-to-end pose gradient through the render."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import full_parity, to_np
from oracle import actors as oa

pytestmark = pytest.mark.gpu


def _ulp_diff(a, b):
    a = np.ascontiguousarray(a, np.float32).view(np.int32).astype(np.int64)
    b = np.ascontiguousarray(b, np.float32).view(np.int32).astype(np.int64)
    return np.abs(a - b)


def _scene(seed=0, n_bg=3000, n_actors=12, per_actor=250, shuffle=False, bad_ids=True):
    rng = np.random.default_rng(seed)
    g, s = synth.scene_pinhole_small(seed, n=n_bg, width=160, height=120, f=110.0)
    g, ids, poses = synth.actors(rng, g, n_actors, per_actor, [[-2.5, 2.5], [-1.5, 1.5], [4, 9]], up_axis=1,
                                 scale=(0.02, 0.15))
    poses[:, :4] *= rng.uniform(0.5, 2.0, (n_actors, 1)).astype(np.float32)   # unnormalised quaternions
    if bad_ids:
        ids[rng.choice(n_bg, 11, replace=False)] = n_actors + 5                 # outside the table: background
    if shuffle:
        perm = rng.permutation(len(ids))
        g, ids = synth.permute(g, perm), ids[perm]
    return g, s, ids, poses


def _gpu_world(g_np, ids, poses):
    import paper_2510_12901_amd as ut
    g = ut.GaussianSet.from_numpy(g_np)
    a = torch.as_tensor(ids, device="cuda")
    w = ut.actor_transform(g, a, ut.actor_poses(poses).cuda())
    torch.cuda.synchronize()
    return g, a, w


@pytest.mark.parametrize("shuffle", [False, True])
def test_actor_transform_matches_oracle(shuffle):
    g_np, _, ids, poses = _scene(1, shuffle=shuffle)
    _, _, w = _gpu_world(g_np, ids, poses)
    ref = oa.actor_transform_f32(g_np, ids, poses)
    for k in ("mean", "quat"):
        d = _ulp_diff(to_np(getattr(w, k)), ref[k])
        assert d.max() <= 1 and (d > 0).mean() < 1e-4, (k, d.max(), (d > 0).sum())
    bg = (ids < 0) | (ids >= len(poses))
    assert np.array_equal(to_np(w.mean)[:, bg], g_np["mean"][:, bg])
    assert np.array_equal(to_np(w.quat)[:, bg], g_np["quat"][:, bg])


def test_actor_scene_render_parity():
    """The GPU's world-frame set equals the oracle's, and that set renders to parity."""
    g_np, s, ids, poses = _scene(2)
    _, _, w = _gpu_world(g_np, ids, poses)
    ref = oa.actor_transform_f32(g_np, ids, poses)
    assert _ulp_diff(to_np(w.mean), ref["mean"]).max() <= 1
    errs, n_ex, gp, oo, _ = full_parity(ref, s)
    print("actors max-abs", errs, "excluded rays", n_ex, "pairs", gp["n_pairs"])
    assert gp["n_pairs"] > 1000 and n_ex <= 0.001 * oo["alpha"].size


@pytest.mark.parametrize("shuffle", [False, True])
def test_actor_backward_matches_oracle(shuffle):
    """Wavefronts of one actor reduce before their atomics; shuffled particles take the
    per-lane path; both against the oracle's adjoint."""
    import paper_2510_12901_amd as ut
    g_np, _, ids, poses = _scene(3, shuffle=shuffle)
    g, a, _ = _gpu_world(g_np, ids, poses)
    rng = np.random.default_rng(4)
    n = len(ids)
    gm = rng.standard_normal((3, n)).astype(np.float32)
    gq = rng.standard_normal((4, n)).astype(np.float32)
    dm, dq, dp = ut.actor_transform_backward(g, a, ut.actor_poses(poses).cuda(), torch.as_tensor(gm, device="cuda"),
                                             torch.as_tensor(gq, device="cuda"))
    torch.cuda.synchronize()
    rm, rq, rp = oa.actor_transform_backward(g_np, ids, poses, gm, gq)
    np.testing.assert_allclose(to_np(dm), rm, rtol=2e-7, atol=2e-7 * np.abs(rm).max())
    np.testing.assert_allclose(to_np(dq), rq, rtol=2e-7, atol=2e-7 * np.abs(rq).max())
    np.testing.assert_allclose(to_np(dp), rp, rtol=1e-10, atol=1e-10 * np.abs(rp).max())
    # no pose gradient requested: the object-frame gradients are unchanged
    dm2, dq2, dp2 = ut.actor_transform_backward(g, a, ut.actor_poses(poses).cuda(),
                                                torch.as_tensor(gm, device="cuda"), torch.as_tensor(gq, device="cuda"),
                                                pose_grad=False)
    assert dp2 is None and torch.equal(dm, dm2) and torch.equal(dq, dq2)


def test_pose_gradient_through_the_render():
    """loss(render(transform(object set, poses))) differentiated by autograd through both hand-
    written adjoints, against the oracle's render adjoint chained into its transform adjoint
    (relative 1e-3 with a floor of 1e-3 x the RMS, as for the render's own adjoint)."""
    import paper_2510_12901_amd as ut
    g_np, s_np, ids, poses = _scene(5, n_bg=1500, n_actors=6, per_actor=200, bad_ids=False)
    g = ut.GaussianSet.from_numpy(g_np)
    s = ut.Sensor(s_np)
    a = torch.as_tensor(ids, device="cuda")
    P = torch.as_tensor(poses, device="cuda").requires_grad_(True)
    mean = g.mean.clone().requires_grad_(True)
    gw = ut.transform_differentiable(g.with_params(mean, g.quat, g.log_scale, g.opacity_logit, g.feat), a, P)
    feat, depth, alpha, _ = ut.render_differentiable(gw, s)
    target = torch.as_tensor(synth.l1_target(7, (3, s.n_rays)), device="cuda")
    loss = (feat - target).abs().mean() + 0.01 * depth.mean()
    loss.backward()
    torch.cuda.synchronize()
    # oracle: render the oracle's world set, adjoint of the render, then of the transform
    w = oa.actor_transform_f32(g_np, ids, poses)
    _, ol, oo = oracle.render(w, s_np)
    R = s.n_rays
    up = dict(feat=(np.sign(oo["feat"] - to_np(target).astype(np.float64)) / (3 * R)).astype(np.float32).astype(np.float64),
              depth=np.full(R, np.float64(np.float32(0.01 / R))))
    rg = oracle.backward(w, s_np, ol, up)
    rm, _, rp = oa.actor_transform_backward(g_np, ids, poses, rg["mean"], rg["quat"])
    for name, got, ref in (("pose", to_np(P.grad), rp), ("mean", to_np(mean.grad), rm)):
        got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
        rms = np.sqrt(np.mean(ref ** 2)) + 1e-300
        err = np.abs(got - ref) / (np.abs(ref) + 1e-3 * rms)
        assert err.max() <= 1e-3, (name, float(err.max()))
    assert np.abs(rp).max() > 0
