"""Every entry point of the oracle on small seeded scenes (camera, fisheye, LiDAR with culling,
beam divergence, moving sensors, adjoint, finite differences).  Run by test_sanitizers.py in a
child process against an AddressSanitizer + UndefinedBehaviorSanitizer build of the oracle."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

assert os.environ.get("UTORACLE_LIB"), "run through test_sanitizers.py"
scenes = [synth.scene_pinhole_small(0, n=300),
          synth.scene_fisheye(3, n=2000, width=64, height=48),
          synth.scene_lidar(4, n=2000, n_beams=16, n_az=128, n_phi=4, max_per_tile=32),
          synth.scene_lidar(5, n=2000, n_beams=16, n_az=128, n_phi=4, max_per_tile=32, cull=False)]
g, s = synth.scene_lidar(6, n=1500, n_beams=16, n_az=128, n_phi=4, max_per_tile=32)
s["beam_divergence"] = 0.02
scenes.append((g, s))
g, s = synth.scene_pinhole_small(1, n=300)
scenes.append((g, synth.rolling_shutter(s, synth.yaw_camera_pose(0.1), s["origin"] + np.float32([0.3, 0, 0]))))
for g, s in scenes:
    g["mean"] *= np.float32(0.1) if s["kind"] == 2 else np.float32(1)
    op, ol, oo = oracle.render(g, s)
    rng = np.random.default_rng(0)
    R = oracle.OracleSensor(s).n_rays
    up = {"feat": rng.standard_normal((3, R)), "depth": rng.standard_normal(R), "alpha": rng.standard_normal(R)}
    if s["kind"] == 2:
        up["drop"] = rng.standard_normal(R)
    oracle.backward(g, s, ol, up)
    vis = np.nonzero(op["count"])[0][:3]
    if len(vis):
        oracle.fd_grad(g, s, ol, up, vis, h=1e-4)
    oracle.composite_rays(g, s, ol, np.arange(0, R, 7))
    oracle.bin_pairs(oracle.OracleSensor(s), op["rect"], op["count"], op["key"])
be = synth.beams_uniform(np.random.default_rng(1), 32)
oracle.lidar_tiling(be, 512, 8, 32)
print("ok")
