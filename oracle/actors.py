"""Rigid actor transforms of the scene graph (Sec. 3.1, scene representation): FP64 oracle.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by ``tests/`` and never by
the product package.

The paper assigns every particle either to the static background or to one dynamic object.
An object's particles keep their means and covariances in the object's own frame; at render
time the object's SE(3) pose for the timestamp maps them to the world.  Written out:

    mu_w = R_a mu + t_a,    Sigma_w = R_a Sigma R_a^T,

so with Sigma = R(q) S S^T R(q)^T the world rotation is R_a R(q), i.e. the quaternion
q_w = q_a * q (Hamilton product, (w, x, y, z) order).  Scale, opacity and the feature
coefficients are left as they are (the paper moves means and covariances only).

Pose layout: [n_actors, 7] = (qw, qx, qy, qz, tx, ty, tz); the pose quaternion is normalised
before use.  actor[i] = -1 (or any id outside [0, n_actors)) is background: unchanged.
"""
from __future__ import annotations

import numpy as np


def quat_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product of quaternions stored as rows (w, x, y, z) of [4, n] arrays."""
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrices [n, 3, 3] of unit quaternions [4, n] (w, x, y, z)."""
    w, x, y, z = q
    return np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
                     np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
                     np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def _members(actor, n_actors):
    actor = np.asarray(actor, np.int64)
    return (actor >= 0) & (actor < n_actors), actor


def actor_transform(g: dict, actor, poses) -> dict:
    """World-frame particle set: means and quaternions of actor particles moved by their pose
    (float64; every other entry of ``g`` is passed through)."""
    poses = np.asarray(poses, np.float64).reshape(-1, 7)
    mean = np.asarray(g["mean"], np.float64).copy()
    quat = np.asarray(g["quat"], np.float64).copy()
    on, actor = _members(actor, poses.shape[0])
    idx = np.nonzero(on)[0]
    if len(idx):
        p = poses[actor[idx]]
        qa = (p[:, :4] / np.linalg.norm(p[:, :4], axis=1, keepdims=True)).T
        R = quat_to_rot(qa)
        mean[:, idx] = np.einsum("nij,jn->in", R, mean[:, idx]) + p[:, 4:].T
        quat[:, idx] = quat_mul(qa, quat[:, idx])
    out = dict(g)
    out["mean"], out["quat"] = mean, quat
    return out


def actor_transform_f32(g: dict, actor, poses) -> dict:
    """The world-frame set rounded once to float32, as a render takes it."""
    w = actor_transform(g, actor, poses)
    w["mean"] = w["mean"].astype(np.float32)
    w["quat"] = w["quat"].astype(np.float32)
    return w


def actor_transform_backward(g: dict, actor, poses, d_mean_w, d_quat_w):
    """Adjoint of ``actor_transform``: given dL/d(world mean) [3, n] and dL/d(world quaternion)
    [4, n], returns dL/d(object mean), dL/d(object quaternion) and dL/d(pose) [n_actors, 7]
    (with respect to the raw pose quaternion, before its normalisation, and the translation)."""
    poses = np.asarray(poses, np.float64).reshape(-1, 7)
    n_act = poses.shape[0]
    mean = np.asarray(g["mean"], np.float64)
    quat = np.asarray(g["quat"], np.float64)
    dmw = np.asarray(d_mean_w, np.float64)
    dqw = np.asarray(d_quat_w, np.float64)
    d_mean, d_quat = dmw.copy(), dqw.copy()
    d_pose = np.zeros((n_act, 7))
    on, actor = _members(actor, n_act)
    idx = np.nonzero(on)[0]
    if not len(idx):
        return d_mean, d_quat, d_pose
    p = poses[actor[idx]]
    qn = np.linalg.norm(p[:, :4], axis=1)
    qa = (p[:, :4] / qn[:, None]).T
    R = quat_to_rot(qa)
    mu, q, gm, gq = mean[:, idx], quat[:, idx], dmw[:, idx], dqw[:, idx]
    # mu_w = R mu + t: dL/dmu = R^T g, dL/dt = g, dL/dR = g mu^T
    d_mean[:, idx] = np.einsum("nji,jn->in", R, gm)
    dR = np.einsum("in,jn->nij", gm, mu)
    # q_w = q_a * q is linear in either factor: the adjoint of multiplying by q_a on the
    # left is multiplying by conj(q_a) on the left, the adjoint of multiplying q_a on the
    # right by q is multiplying by conj(q) on the right
    conj = lambda v: v * np.array([1.0, -1.0, -1.0, -1.0])[:, None]
    d_quat[:, idx] = quat_mul(conj(qa), gq)
    dqa = quat_mul(gq, conj(q))
    # dL/dq_k = sum_ij dL/dR_ij dR_ij/dq_k with the partial derivatives of the polynomial R(q)
    w, x, y, z = qa
    o = np.zeros_like(w)
    J = 2 * np.stack([
        np.stack([np.stack([o, -z, y], -1), np.stack([z, o, -x], -1), np.stack([-y, x, o], -1)], -2),
        np.stack([np.stack([o, y, z], -1), np.stack([y, -2 * x, -w], -1), np.stack([z, w, -2 * x], -1)], -2),
        np.stack([np.stack([-2 * y, x, w], -1), np.stack([x, o, z], -1), np.stack([-w, z, -2 * y], -1)], -2),
        np.stack([np.stack([-2 * z, -w, x], -1), np.stack([w, -2 * z, y], -1), np.stack([x, y, o], -1)], -2)])
    dqa = dqa + np.einsum("knij,nij->kn", J, dR)
    # normalisation q_hat = q / |q|
    dqa = (dqa - qa * np.sum(qa * dqa, axis=0)) / qn
    for k in range(4):
        np.add.at(d_pose[:, k], actor[idx], dqa[k])
    for k in range(3):
        np.add.at(d_pose[:, 4 + k], actor[idx], gm[k])
    return d_mean, d_quat, d_pose
