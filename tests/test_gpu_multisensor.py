"""Parity of the benchmarked multi-sensor frame itself: 2,000,000 particles stored in Z-order
on the device, 4 pinhole 1920x1080 + 2 fisheye 1920x1280 + 1 LiDAR 128x2048 at random poses,
each sensor on its own stream with the pair total kept on the device (the launch
configuration the benchmark times).  Per sensor: depth keys bit-exact, counts and rects equal
to the oracle's projection, every tile list bit-exact against the oracle's binning, and 4,096
sampled rays within 1e-4 of the oracle's per-ray compositing."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import AMBIG, TOL, same_ranges, to_np
from test_gpu_layout import _morton_np

pytestmark = pytest.mark.gpu


def _subset_cols(g, perm):
    out = dict(g)
    for k in ("mean", "quat", "log_scale", "opacity_logit", "feat"):
        out[k] = np.ascontiguousarray(g[k][..., perm])
    return out


def test_multisensor_frame_parity():
    import paper_2510_12901_amd as ut
    dev = torch.device("cuda:0")
    g_np, gl_np, sensors_np = synth.scene_multisensor(0)
    # the resident set as the benchmark stores it: Z-order of the means (ut_spatial_order +
    # ut_gather_gaussians); the oracle gets the same order from the Morton definition itself
    perm_np = np.argsort(_morton_np(g_np["mean"]), kind="stable")
    g0 = ut.GaussianSet.from_numpy(g_np, dev)
    perm = ut.spatial_order(g0)
    assert np.array_equal(to_np(perm).astype(np.int64), perm_np)
    g = ut.gather(g0, perm)
    gl0 = ut.GaussianSet(g0.mean, g0.quat, g0.log_scale, g0.opacity_logit,
                         torch.as_tensor(gl_np["feat"], device=dev), 0, synth.FEAT_LIDAR)
    gl = ut.GaussianSet(g.mean, g.quat, g.log_scale, g.opacity_logit, ut.gather(gl0, perm).feat, 0,
                        synth.FEAT_LIDAR)
    del g0, gl0
    sensors = [ut.Sensor(s, dev) for s in sensors_np]
    pipes = [ut.SensorPipeline(gl if s.is_lidar else g, s, state=True) for s in sensors]
    streams = [torch.cuda.Stream(device=dev) for _ in pipes]
    for p, st in zip(pipes, streams):          # a set-up frame sizes the capacities
        p.run(st)
    torch.cuda.synchronize()
    for p in pipes:
        p.set_capacity(int(p.n_pairs * 1.25) + 4096)
        p.clear_overflow()
    for p, st in zip(pipes, streams):          # the measured path: no host round trip
        p.run_device(st)
    torch.cuda.synchronize()
    assert not any(p.overflowed() for p in pipes)

    og = oracle.OracleGaussians(_subset_cols(g_np, perm_np))
    ogl = oracle.OracleGaussians(_subset_cols(gl_np, perm_np))
    n = g.n
    rng = np.random.default_rng(1)
    for si, (pipe, s_np) in enumerate(zip(pipes, sensors_np)):
        os_ = oracle.OracleSensor(s_np)
        lidar = os_.kind == 2
        ogs = ogl if lidar else og
        op = oracle.project(ogs, os_)
        amb = op["margin"] < AMBIG
        key = to_np(pipe.p.key).view(np.uint32)[:n]
        count = to_np(pipe.p.count).view(np.uint32)[:n]
        rect = to_np(pipe.p.rect)[:, :n]
        assert np.array_equal(key, op["key"]), si
        assert np.array_equal(count[~amb], op["count"][~amb]), si
        vis = (~amb) & (op["count"] > 0)
        assert np.array_equal(rect[:, vis], op["rect"][:, vis]), si
        # every tile's list, materialised from the device-count bins, against the oracle's binning
        lists = ut.tile_lists(pipe.p, pipe.sensor, pipe.bins)
        torch.cuda.synchronize()
        ol_g = oracle.bin_pairs(os_, rect, count, key)
        assert lists.n_pairs == ol_g["n_pairs"], si
        assert np.array_equal(to_np(lists.gauss).view(np.uint32)[: lists.n_pairs], ol_g["pair_gauss"]), si
        assert same_ranges(to_np(lists.ranges).view(np.uint32), ol_g["ranges"]), si
        del lists
        ol = oracle.bin_pairs(os_, op["rect"], op["count"], op["key"]) if amb.any() else ol_g
        del ol_g
        ids = np.sort(rng.choice(os_.n_rays, 4096, replace=False))
        oo = oracle.composite_rays(ogs, os_, ol, ids)
        keep = oo["margin"] >= AMBIG
        out = pipe.out
        for k in ("feat", "depth", "alpha") + (("drop",) if lidar else ()):
            d = np.abs(np.asarray(to_np(getattr(out, k)), np.float64)[..., ids] - oo[k])[..., keep]
            assert d.max(initial=0) <= TOL, (si, k, float(d.max()))
        n_proc = to_np(out.n_proc).view(np.uint32)
        assert np.array_equal(n_proc[ids][keep], oo["n_proc"][keep]), si
        print(f"sensor {si} kind {os_.kind}: tile pairs {ol['n_pairs']}, ambiguous particles {int(amb.sum())}, "
              f"excluded rays {int((~keep).sum())}")
        del ol, op
