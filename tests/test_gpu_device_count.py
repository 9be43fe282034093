"""The device-count binning path (ut_bin_sort_device): the pair total never leaves the GPU,
launches are sized by a capacity, an over-capacity frame raises a flag and renders nothing."""
import numpy as np
import pytest
import torch

import synth
from test_gpu_parity import _scene

pytestmark = pytest.mark.gpu

KEYS = ("feat", "depth", "alpha", "t_final", "n_proc")


def _pipes(name):
    import paper_2510_12901_amd as ut
    g_np, s_np = _scene(name)
    g = ut.GaussianSet.from_numpy(g_np)
    s = ut.Sensor(s_np)
    return ut, g, s


def _outs(o):
    return {k: getattr(o, k).clone() for k in KEYS if getattr(o, k, None) is not None}


@pytest.mark.parametrize("name", ["pinhole_ragged", "fisheye_small", "lidar_small", "lidar_moving",
                                  "pinhole_rolling_shutter"])
def test_device_count_path_is_bit_identical(name):
    ut, g, s = _pipes(name)
    ref = ut.SensorPipeline(g, s, state=True)
    ref.run()
    torch.cuda.synchronize()
    P = ref.n_pairs
    want = _outs(ref.out)
    dev = ut.SensorPipeline(g, s, state=True)
    dev.set_capacity(int(P * 1.3) + 7)
    for _ in range(2):                                   # two frames in a row on one pipeline
        dev.run_device()
        torch.cuda.synchronize()
        assert not dev.overflowed()
        got = _outs(dev.out)
        for k in want:
            assert torch.equal(want[k], got[k]), (name, k)
        assert torch.equal(ref.bins.ranges, dev.bins.ranges)
        assert torch.equal(ref.bins.gauss[:P], dev.bins.gauss[:P])


def test_over_capacity_raises_the_flag_and_renders_nothing():
    ut, g, s = _pipes("pinhole_ragged")
    ref = ut.SensorPipeline(g, s, state=True)
    ref.run()
    torch.cuda.synchronize()
    P = ref.n_pairs
    dev = ut.SensorPipeline(g, s, state=True)
    dev.set_capacity(P - 1)
    dev.run_device()
    torch.cuda.synchronize()
    assert dev.overflowed()
    assert int(dev.bins.ranges.abs().sum().item()) == 0
    assert float(dev.out.alpha.abs().max().item()) == 0.0
    # the flag stays raised until cleared; with the exact capacity the frame is whole again
    dev.set_capacity(P)
    dev.run_device()
    torch.cuda.synchronize()
    assert dev.overflowed()
    dev.clear_overflow()
    dev.run_device()
    torch.cuda.synchronize()
    assert not dev.overflowed()
    assert torch.equal(ref.out.feat, dev.out.feat) and torch.equal(ref.out.n_proc, dev.out.n_proc)


def test_device_count_path_with_no_pairs():
    ut, g, s = _pipes("pinhole_ragged")
    g_np, s_np = _scene("pinhole_ragged")
    g_np["mean"][2] = -5.0                              # everything behind the camera
    g0 = ut.GaussianSet.from_numpy(g_np)
    dev = ut.SensorPipeline(g0, s, state=True)
    dev.set_capacity(1000)
    dev.run_device()
    torch.cuda.synchronize()
    assert not dev.overflowed()
    assert float(dev.out.alpha.abs().max().item()) == 0.0


def test_frame_graph_replays_match_eager_frames():
    """A frame of four sensors (camera, fisheye, LiDAR, rolling shutter) captured in a graph:
    three replays, each after eager work that overwrites the outputs, every replay bit-identical
    to the eager frame."""
    import paper_2510_12901_amd as ut
    pipes = []
    for name in ("pinhole_ragged", "fisheye_small", "lidar_small", "pinhole_rolling_shutter"):
        _, g, s = _pipes(name)
        p = ut.SensorPipeline(g, s, state=True)
        p.run()
        torch.cuda.synchronize()
        p.set_capacity(int(p.n_pairs * 1.2) + 64)
        pipes.append(p)
    want = [_outs(p.out) for p in pipes]
    fg = ut.FrameGraph(pipes)
    for rep in range(3):
        for p in pipes:                                   # eager work in between: a plain render
            p.run()
            p.out.feat.zero_()
            p.out.alpha.fill_(7.0)
        torch.cuda.synchronize()
        fg.replay()
        torch.cuda.synchronize()
        assert not fg.overflowed()
        for w, p in zip(want, pipes):
            got = _outs(p.out)
            for k in w:
                assert torch.equal(w[k], got[k]), (rep, k)
