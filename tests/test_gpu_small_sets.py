"""Small particle and pair sets: up to 4096 particles the count stage runs in one workgroup, up to
4096 pairs the pair sort does; above that the multi-kernel chains run.  Either way the lists
must be the oracle binning of the GPU's own rects, counts and keys, bit for bit, and the frame
must not depend on which side of the boundary a scene falls."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import gpu_render, same_ranges

pytestmark = pytest.mark.gpu

SMALL = 4096


def _scene(n, seed):
    # 400 x 300 pinhole, 25 x 19 tiles in 4 x 3 super-tiles: particles touch several
    rng = np.random.default_rng(seed)
    mean = np.stack([rng.uniform(-2.5, 2.5, n), rng.uniform(-1.8, 1.8, n), rng.uniform(1.5, 6, n)])
    g = synth.particles(rng, mean, 0.01, 0.25, 0, synth.FEAT_CAMERA)
    return g, synth.pinhole(400, 300, 300.0, 300.0)


def _lists_match_oracle(g, s):
    gp, _ = gpu_render(g, s, moments=False)
    os_ = oracle.OracleSensor(s)
    ol = oracle.bin_pairs(os_, gp["rect"], gp["count"], gp["key"])
    assert gp["n_pairs"] == ol["n_pairs"]
    assert np.array_equal(gp["gauss"], ol["pair_gauss"])
    assert same_ranges(gp["ranges"], ol["ranges"])
    return gp


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (65, 2), (700, 3), (1025, 4), (4095, 5), (4096, 6),
                                    (4097, 7), (9000, 8)])
def test_lists_across_the_single_workgroup_boundaries(n, seed):
    g, s = _scene(n, seed)
    gp = _lists_match_oracle(g, s)
    print(n, "visible", int((gp["count"] > 0).sum()), "super-tile pairs", gp["n_bin_pairs"])


def test_boundaries_are_crossed():
    """The cases above reach both sides of both boundaries (particles and super-tile pairs)."""
    import torch
    import paper_2510_12901_amd as ut
    seen = set()
    for n, seed in [(700, 3), (4095, 5), (9000, 8)]:
        g, s = _scene(n, seed)
        _, bins, _ = ut.render(ut.GaussianSet.from_numpy(g), ut.Sensor(s))
        torch.cuda.synchronize()
        seen.add((n <= SMALL, bins.n_pairs <= SMALL))
    assert (True, True) in seen and (True, False) in seen and (False, False) in seen


def test_frame_is_the_same_on_both_sides_of_the_particle_boundary():
    """4096 particles (one-workgroup count stage) and the same 4096 plus one particle behind the
    camera (multi-kernel count stage): identical lists and outputs."""
    import torch
    import paper_2510_12901_amd as ut
    g, s = _scene(4096, 11)
    extra = synth.subset(g, [0])
    extra["mean"] = extra["mean"].copy()
    extra["mean"][2] = -3.0
    g2 = synth.concat(g, extra)
    outs = []
    S = ut.Sensor(s)
    for gg in (g, g2):
        p, bins, out = ut.render(ut.GaussianSet.from_numpy(gg), S)
        lists = ut.tile_lists(p, S, bins)
        torch.cuda.synchronize()
        outs.append((bins.n_pairs, bins.gauss[:bins.n_pairs].cpu(), bins.ranges.cpu(), lists.gauss[:lists.n_pairs].cpu(),
                     out.feat.cpu(), out.alpha.cpu(), out.n_proc.cpu()))
    a, b = outs
    assert a[0] == b[0]
    for x, y in zip(a[1:], b[1:]):
        assert torch.equal(x, y)


def test_device_count_small_pair_sort_and_overflow():
    """The one-workgroup pair sort with the pair total on the device: identical bins to the
    host-count path within capacity, the overflow flag and empty bins one pair below it."""
    import torch
    import paper_2510_12901_amd as ut
    g, s = _scene(900, 12)
    G, S = ut.GaussianSet.from_numpy(g), ut.Sensor(s)
    ref = ut.SensorPipeline(G, S, state=True)
    ref.run()
    torch.cuda.synchronize()
    P = ref.n_pairs
    assert 0 < P < SMALL
    dev = ut.SensorPipeline(G, S, state=True)
    dev.set_capacity(P)
    dev.run_device()
    torch.cuda.synchronize()
    assert not dev.overflowed()
    assert torch.equal(ref.bins.ranges, dev.bins.ranges)
    assert torch.equal(ref.bins.gauss[:P], dev.bins.gauss[:P])
    assert torch.equal(ref.out.feat, dev.out.feat)
    dev2 = ut.SensorPipeline(G, S, state=True)
    dev2.set_capacity(P - 1)
    dev2.run_device()
    torch.cuda.synchronize()
    assert dev2.overflowed()
    assert int(dev2.bins.ranges.abs().sum().item()) == 0
    assert float(dev2.out.alpha.abs().max().item()) == 0.0


def test_device_count_small_pair_sort_bounded_by_the_super_tiles():
    """128 x 96 camera (one super-tile), 1,000 particles, a large capacity: the pair total is
    bounded by particles x super-tiles, so the one-workgroup sort runs; bins equal the
    host-count path's."""
    import torch
    import paper_2510_12901_amd as ut
    g, s = synth.scene_pinhole_small(0)
    G, S = ut.GaussianSet.from_numpy(g), ut.Sensor(s)
    ref = ut.SensorPipeline(G, S, state=True)
    ref.run()
    torch.cuda.synchronize()
    P = ref.n_pairs
    dev = ut.SensorPipeline(G, S, state=True)
    dev.set_capacity(100_000)
    for _ in range(2):
        dev.run_device()
        torch.cuda.synchronize()
        assert not dev.overflowed()
        assert torch.equal(ref.bins.ranges, dev.bins.ranges)
        assert torch.equal(ref.bins.gauss[:P], dev.bins.gauss[:P])
        assert torch.equal(ref.out.feat, dev.out.feat) and torch.equal(ref.out.n_proc, dev.out.n_proc)
