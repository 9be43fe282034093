"""Seeded synthetic inputs for the UT Gaussian rasterizer: particle sets, sensors, ray tables.

This module is shared by the GPU path, the oracle and the benchmark. It holds no step of
the rendering method: it only draws random particles from stated distributions and builds
sensor descriptions and their ray tables (the rays r(t) = o + t d that the renderer takes as
input, Sec. 3.2 "Volume Rendering").  Ray tables are built in float64 and rounded to
float32 once, so every consumer sees the same float32 rays.

Conventions
-----------
* Gaussians are structure-of-arrays float32:
  ``mean[3,N]``, ``quat[4,N]`` (w,x,y,z, unnormalised allowed), ``log_scale[3,N]``,
  ``opacity_logit[N]``, ``feat[K,3,N]`` with K=(deg+1)^2 SH coefficients per channel.
* ``feat_kind`` 0 = camera colour (the renderer evaluates SH, adds 0.5 and clamps at 0),
  1 = LiDAR features (intensity, hit logit, drop logit), used raw.
* A sensor is a dict.  ``R_sw`` (float32 3x3) maps world to sensor axes, ``origin``
  (float32 3) is the sensor position in the world.  Camera axes: x right, y down,
  z forward.  LiDAR axes: x forward, y left, z up.
* ``ray_dir`` is float32 ``[3, R]`` in the world frame, unit length; an all-zero column
  marks a pixel with no ray (fisheye corners beyond the field of view).
  Camera ray index = y*W + x through the pixel centre (x+0.5, y+0.5).
  LiDAR ray index = b*n_az + a, beam b at elevation ``beam_elev[b]`` (sorted ascending),
  azimuth 2*pi*a/n_az.
"""
from __future__ import annotations

import numpy as np

PINHOLE, FISHEYE, LIDAR, ORTHO = 0, 1, 2, 3
FEAT_CAMERA, FEAT_LIDAR = 0, 1

# A degree-0 SH coefficient k contributes k * Y00 with Y00 = 1/(2 sqrt(pi)); drawing the
# coefficient as value * 2 sqrt(pi) makes the evaluated degree-0 feature equal `value`.
DC_SCALE = 2.0 * np.sqrt(np.pi)


# ----------------------------------------------------------------------------- particles
def unit_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotations: normalised 4D standard normals, (w,x,y,z) rows."""
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q.astype(np.float32)


def logit(p: np.ndarray) -> np.ndarray:
    return np.log(p / (1.0 - p))


def particles(rng, mean, scale_lo, scale_hi, n_sh_deg, feat_kind,
              dc=None, hi_sigma=0.1, opacity=(0.05, 0.95)):
    """Common particle attributes around given means.

    ``dc``: float array [3,N] of the desired degree-0 feature values (converted to
    coefficients with DC_SCALE); higher-order coefficients are N(0, hi_sigma).
    """
    n = mean.shape[1]
    K = (n_sh_deg + 1) ** 2
    quat = unit_quaternions(rng, n)
    log_scale = rng.uniform(np.log(scale_lo), np.log(scale_hi), (3, n))
    op = rng.uniform(opacity[0], opacity[1], n)
    feat = np.zeros((K, 3, n), np.float64)
    if dc is None:
        dc = rng.uniform(0.0, 1.0, (3, n))
    feat[0] = dc
    if K > 1:
        feat[1:] = rng.normal(0.0, hi_sigma, (K - 1, 3, n))
    return dict(mean=mean.astype(np.float32), quat=quat,
                log_scale=log_scale.astype(np.float32),
                opacity_logit=logit(op).astype(np.float32),
                feat=feat.astype(np.float32), sh_degree=n_sh_deg, feat_kind=feat_kind)


def camera_rgb_dc(rgb: np.ndarray) -> np.ndarray:
    """DC coefficients whose evaluated camera colour (f + 0.5) equals ``rgb``."""
    return (rgb - 0.5) * DC_SCALE


def lidar_feat(rng, n):
    """LiDAR degree-0 features: intensity U[0,1], hit logit 0, drop logit N(0,1)."""
    vals = np.zeros((3, n))
    vals[0] = rng.uniform(0.0, 1.0, n)
    vals[2] = rng.standard_normal(n)
    return (vals * DC_SCALE).astype(np.float32)[None]      # [1,3,N]


def subset(g: dict, idx) -> dict:
    out = dict(g)
    for k in ("mean", "quat", "log_scale"):
        out[k] = np.ascontiguousarray(g[k][:, idx])
    out["opacity_logit"] = np.ascontiguousarray(g["opacity_logit"][idx])
    out["feat"] = np.ascontiguousarray(g["feat"][:, :, idx])
    return out


def permute(g: dict, perm) -> dict:
    return subset(g, np.asarray(perm))


def concat(a: dict, b: dict) -> dict:
    """Two particle sets of the same SH degree and feature kind, one after the other."""
    out = dict(a)
    for k in ("mean", "quat", "log_scale"):
        out[k] = np.ascontiguousarray(np.concatenate([a[k], b[k]], 1))
    out["opacity_logit"] = np.concatenate([a["opacity_logit"], b["opacity_logit"]])
    out["feat"] = np.ascontiguousarray(np.concatenate([a["feat"], b["feat"]], 2))
    return out


def actors(rng, g_background: dict, n_actors: int, per_actor: int, region, box=(4.5, 1.8, 1.5),
           up_axis=2, scale=(0.02, 0.3), feat=None):
    """Dynamic objects appended to a background set: per actor, ``per_actor`` particles in a
    car-sized box of the object's own frame (centred on its origin), and an object-to-world
    pose (yaw about ``up_axis``, centre uniform in ``region`` = [[lo, hi]] * 3).

    Returns (particles, actor ids [N] int32 with -1 for the background, poses [n_actors, 7]
    float32 = (qw, qx, qy, qz, tx, ty, tz)).  The background keeps its order and comes first."""
    n = n_actors * per_actor
    half = np.asarray(box, np.float64) / 2
    mean = np.stack([rng.uniform(-h, h, n) for h in half])
    if up_axis != 2:
        mean = np.roll(mean, up_axis - 2, axis=0)
    kind, deg = g_background["feat_kind"], g_background["sh_degree"]
    obj = particles(rng, mean, scale[0], scale[1], deg, kind)
    if feat is not None:
        obj["feat"] = feat(rng, n)
    yaw = rng.uniform(0, 2 * np.pi, n_actors)
    q = np.zeros((n_actors, 4))
    q[:, 0] = np.cos(yaw / 2)
    q[:, 1 + up_axis] = np.sin(yaw / 2)
    region = np.asarray(region, np.float64)
    t = np.stack([rng.uniform(lo, hi, n_actors) for lo, hi in region], 1)
    poses = np.concatenate([q, t], 1).astype(np.float32)
    ids = np.concatenate([np.full(g_background["mean"].shape[1], -1), np.repeat(np.arange(n_actors), per_actor)])
    return concat(g_background, obj), ids.astype(np.int32), poses


# ----------------------------------------------------------------------------- poses
def yaw_camera_pose(yaw: float) -> np.ndarray:
    """World (z up) -> camera axes (x right, y down, z forward) looking along yaw."""
    fwd = np.array([np.cos(yaw), np.sin(yaw), 0.0])
    right = np.array([np.sin(yaw), -np.cos(yaw), 0.0])
    down = np.array([0.0, 0.0, -1.0])
    return np.stack([right, down, fwd]).astype(np.float32)


def yaw_lidar_pose(yaw: float) -> np.ndarray:
    c, s = np.cos(yaw), np.sin(yaw)
    # rows are the sensor axes expressed in the world frame
    return np.array([[c, s, 0.0], [-s, c, 0.0], [0.0, 0.0, 1.0]], np.float32)


def random_ball(rng, radius: float) -> np.ndarray:
    while True:
        p = rng.uniform(-radius, radius, 3)
        if np.dot(p, p) <= radius * radius:
            return p


# ----------------------------------------------------------------------------- sensors
def _to_world(R_sw, d_sensor):
    d = R_sw.astype(np.float64).T @ d_sensor
    n = np.linalg.norm(d, axis=0, keepdims=True)
    d = np.where(n > 0, d / np.where(n > 0, n, 1.0), 0.0)
    return np.ascontiguousarray(d.astype(np.float32))


def _add_motion(desc, d_sensor, times, R_sw1, origin1, rs_iters=3):
    """Moving sensor: pose (R_sw, origin) at frame time 0 and (R_sw1, origin1) at 1; ray i,
    captured at times[i], gets the world direction R(t_i)^T d_i and the origin o(t_i), with the
    origin linear in t and the rotation spherically interpolated (scipy's Slerp)."""
    from scipy.spatial.transform import Rotation, Slerp
    R0 = np.asarray(desc["R_sw"], np.float32).astype(np.float64)
    R1 = np.asarray(R_sw1, np.float32).astype(np.float64)
    o0 = np.asarray(desc["origin"], np.float32).astype(np.float64)
    o1 = np.asarray(origin1, np.float32).astype(np.float64)
    slerp = Slerp([0.0, 1.0], Rotation.from_matrix(np.stack([R0, R1])))
    Rt = slerp(np.clip(times, 0.0, 1.0)).as_matrix()                 # [R,3,3] world->sensor
    d = np.einsum("rji,jr->ir", Rt, d_sensor)                           # R^T d per ray
    n = np.linalg.norm(d, axis=0, keepdims=True)
    d = np.where(n > 0, d / np.where(n > 0, n, 1.0), 0.0)
    d[:, ~np.any(d_sensor != 0, axis=0)] = 0.0
    org = (1.0 - times)[None, :] * o0[:, None] + times[None, :] * o1[:, None]
    desc.update(moving=1, R_sw1=np.asarray(R_sw1, np.float32), origin1=np.asarray(origin1, np.float32),
                ray_dir=np.ascontiguousarray(d.astype(np.float32)),
                ray_org=np.ascontiguousarray(org.astype(np.float32)), rs_iters=rs_iters)
    return desc


def rolling_shutter(desc, R_sw1, origin1, rs_iters=3):
    """Camera with rolling shutter: rows read out top to bottom, row r at frame time
    (r + 0.5) / H.  desc is a static camera from pinhole() / fisheye() holding the pose at t=0."""
    W, H = desc["width"], desc["height"]
    ys = np.repeat(np.arange(H), W)
    times = (ys + 0.5) / H
    d_sensor = np.asarray(desc["R_sw"], np.float32).astype(np.float64) @ desc["ray_dir"].astype(np.float64)
    d_sensor[:, ~np.any(desc["ray_dir"] != 0, axis=0)] = 0.0
    return _add_motion(dict(desc), d_sensor, times, R_sw1, origin1, rs_iters)


def spinning(desc, R_sw1, origin1, rs_iters=3):
    """Spinning LiDAR in motion: azimuth column a fired at frame time a / n_az."""
    n_az = desc["n_az"]
    times = np.tile(np.arange(n_az) / n_az, desc["n_beams"])
    d_sensor = np.asarray(desc["R_sw"], np.float32).astype(np.float64) @ desc["ray_dir"].astype(np.float64)
    return _add_motion(dict(desc), d_sensor, times, R_sw1, origin1, rs_iters)


def pinhole(width, height, fx, fy, cx=None, cy=None, R_sw=None, origin=None,
            near=0.1, kind=PINHOLE):
    cx = width / 2.0 if cx is None else cx
    cy = height / 2.0 if cy is None else cy
    R_sw = np.eye(3, dtype=np.float32) if R_sw is None else np.asarray(R_sw, np.float32)
    origin = np.zeros(3, np.float32) if origin is None else np.asarray(origin, np.float32)
    ys, xs = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    u = (xs.ravel() + 0.5 - cx) / fx
    v = (ys.ravel() + 0.5 - cy) / fy
    if kind == ORTHO:
        # parallel rays along +z; the per-ray origin offset is not modelled, so ORTHO
        # sensors are for projection tests only
        d = np.stack([np.zeros_like(u), np.zeros_like(u), np.ones_like(u)])
    else:
        d = np.stack([u, v, np.ones_like(u)])
    return dict(kind=kind, width=width, height=height, tile=16, fx=float(fx), fy=float(fy),
                cx=float(cx), cy=float(cy), k=[0.0] * 4, theta_max=0.0, near=near,
                R_sw=R_sw, origin=origin, ray_dir=_to_world(R_sw, d))


def fisheye_distortion(rng, theta_max, lo=-0.05, hi=0.05, grid=4096):
    """Draw k1..k4 until the equidistant distortion theta*(1+k1 t^2+...) is increasing."""
    th = np.linspace(0.0, theta_max, grid)
    while True:
        k = rng.uniform(lo, hi, 4)
        slope = 1 + 3 * k[0] * th**2 + 5 * k[1] * th**4 + 7 * k[2] * th**6 + 9 * k[3] * th**8
        if np.all(slope > 0):
            return k


def fisheye(width, height, k, theta_max_deg=95.0, R_sw=None, origin=None, near=0.1):
    """Equidistant fisheye with polynomial distortion; focal chosen so the horizontal
    field of view spans 2*theta_max across the image width."""
    R_sw = np.eye(3, dtype=np.float32) if R_sw is None else np.asarray(R_sw, np.float32)
    origin = np.zeros(3, np.float32) if origin is None else np.asarray(origin, np.float32)
    k = np.asarray(k, np.float64)
    tmax = np.deg2rad(theta_max_deg)

    def dist(t):
        t2 = t * t
        return t * (1 + t2 * (k[0] + t2 * (k[1] + t2 * (k[2] + t2 * k[3]))))

    def ddist(t):
        t2 = t * t
        return 1 + t2 * (3 * k[0] + t2 * (5 * k[1] + t2 * (7 * k[2] + t2 * 9 * k[3])))

    f = (width / 2.0) / dist(tmax)
    cx, cy = width / 2.0, height / 2.0
    ys, xs = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    du = (xs.ravel() + 0.5 - cx) / f
    dv = (ys.ravel() + 0.5 - cy) / f
    rd = np.hypot(du, dv)
    # Newton inversion of the (monotone) distortion polynomial; beyond theta_max no ray
    th = np.minimum(rd, tmax)
    for _ in range(60):
        step = (dist(th) - rd) / ddist(th)
        th = np.clip(th - step, 0.0, 2 * tmax)
        if np.abs(step).max() < 1e-15:
            break
    valid = (rd <= dist(tmax))
    s = np.where(rd > 0, np.sin(th) / np.where(rd > 0, rd, 1.0), 0.0)
    d = np.stack([du * s, dv * s, np.cos(th)])
    d[:, ~valid] = 0.0
    return dict(kind=FISHEYE, width=width, height=height, tile=16, fx=float(f), fy=float(f),
                cx=cx, cy=cy, k=[float(x) for x in k], theta_max=float(tmax), near=near,
                R_sw=R_sw, origin=origin, ray_dir=_to_world(R_sw, d))


def lidar(beam_elev, n_az, R_sw=None, origin=None, near=0.1, n_phi=16, max_per_tile=32,
          cull=True, cull_az=1600, cull_el_per_tile=8):
    R_sw = np.eye(3, dtype=np.float32) if R_sw is None else np.asarray(R_sw, np.float32)
    origin = np.zeros(3, np.float32) if origin is None else np.asarray(origin, np.float32)
    be = np.sort(np.asarray(beam_elev, np.float32))
    el = be.astype(np.float64)[:, None]
    az = (2.0 * np.pi * np.arange(n_az) / n_az)[None, :]
    d = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az),
                  np.broadcast_to(np.sin(el), (len(be), n_az))]).reshape(3, -1)
    return dict(kind=LIDAR, beam_elev=be, n_beams=len(be), n_az=n_az, near=near,
                n_phi=n_phi, max_per_tile=max_per_tile, cull=cull, cull_az=cull_az,
                cull_el=cull_el_per_tile * n_phi, R_sw=R_sw, origin=origin,
                ray_dir=_to_world(R_sw, d))


def n_rays(sensor) -> int:
    return sensor["ray_dir"].shape[1]


# ----------------------------------------------------------------------------- workloads
UT_ABK = (1.0, 2.0, 0.0)   # unscented-transform alpha, beta, kappa of every workload


def scene_pinhole_small(seed=0, n=1000, width=128, height=96, f=100.0):
    """1,000 Gaussians in front of a 128x96 pinhole (fx=fy=100), SH degree 0."""
    rng = np.random.default_rng(seed)
    mean = np.stack([rng.uniform(-2, 2, n), rng.uniform(-1.5, 1.5, n), rng.uniform(2, 6, n)])
    rgb = rng.uniform(0.0, 1.0, (3, n))
    g = particles(rng, mean, 0.01, 0.1, 0, FEAT_CAMERA, dc=camera_rgb_dc(rgb))
    return g, pinhole(width, height, f, f)


def box_means(rng, n, half=(50.0, 5.0, 50.0)):
    return np.stack([rng.uniform(-h, h, n) for h in half])


def scene_fisheye(seed=0, n=500_000, width=1920, height=1280):
    """Gaussians in a 100x10x100 m box (camera frame, y down) around a 190-degree fisheye."""
    rng = np.random.default_rng(seed)
    mean = box_means(rng, n)
    g = particles(rng, mean, 0.02, 1.0, 3, FEAT_CAMERA)
    k = fisheye_distortion(rng, np.deg2rad(95.0))
    return g, fisheye(width, height, k)


def beams_uniform(rng, n_beams=128, lo_deg=-25.0, hi_deg=15.0):
    return np.sort(np.deg2rad(rng.uniform(lo_deg, hi_deg, n_beams))).astype(np.float32)


def scene_lidar(seed=0, n=300_000, n_beams=128, n_az=2048, n_phi=16, max_per_tile=32,
                cull=True):
    """Spinning LiDAR at the origin; means uniform in range [1,200] m, azimuth, height."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(1.0, 200.0, n)
    phi = rng.uniform(0.0, 2 * np.pi, n)
    z = rng.uniform(-3.0, 10.0, n)
    mean = np.stack([r * np.cos(phi), r * np.sin(phi), z])
    g = particles(rng, mean, 0.02, 1.0, 0, FEAT_LIDAR)
    g["feat"] = lidar_feat(rng, n)
    sensor = lidar(beams_uniform(rng, n_beams), n_az, n_phi=n_phi,
                   max_per_tile=max_per_tile, cull=cull)
    return g, sensor


def scene_pinhole_large(seed=0, n=1_000_000, width=1920, height=1080, f=1200.0):
    rng = np.random.default_rng(seed)
    mean = box_means(rng, n)
    g = particles(rng, mean, 0.02, 1.0, 3, FEAT_CAMERA)
    return g, pinhole(width, height, f, f)


def l1_target(seed, shape):
    """Seeded target image U[0,1] for the L1 upstream loss."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, shape).astype(np.float32)


def scene_multisensor(seed=0, n=2_000_000, n_cameras_pinhole=4, n_cameras_fisheye=2,
                      with_lidar=True, pinhole_size=(1920, 1080), fisheye_size=(1920, 1280),
                      lidar_beams=128, lidar_az=2048):
    """Resident scene (world z up) with camera SH and LiDAR features per Gaussian, and one
    frame's sensor rig: pinhole and fisheye cameras plus a spinning LiDAR, each at a random
    position within 2 m of the origin with a random yaw."""
    rng = np.random.default_rng(seed)
    mean = box_means(rng, n, half=(50.0, 50.0, 5.0))
    g = particles(rng, mean, 0.02, 1.0, 3, FEAT_CAMERA)
    glidar = dict(g)
    glidar["feat"] = lidar_feat(rng, n)
    glidar["sh_degree"] = 0
    glidar["feat_kind"] = FEAT_LIDAR
    sensors = []
    for _ in range(n_cameras_pinhole):
        sensors.append(pinhole(*pinhole_size, 1200.0, 1200.0, R_sw=yaw_camera_pose(rng.uniform(0, 2 * np.pi)),
                               origin=random_ball(rng, 2.0)))
    k = fisheye_distortion(rng, np.deg2rad(95.0))
    for _ in range(n_cameras_fisheye):
        sensors.append(fisheye(*fisheye_size, k, R_sw=yaw_camera_pose(rng.uniform(0, 2 * np.pi)),
                               origin=random_ball(rng, 2.0)))
    if with_lidar:
        sensors.append(lidar(beams_uniform(rng, lidar_beams), lidar_az,
                             R_sw=yaw_lidar_pose(rng.uniform(0, 2 * np.pi)),
                             origin=random_ball(rng, 2.0)))
    return g, glidar, sensors
