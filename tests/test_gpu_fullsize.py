"""Full-size workloads in the launch configuration the benchmark times: lists compared
bit-exactly with the oracle's binning of the GPU projection, and 4,096 sampled rays per
workload compared with the oracle's per-ray compositing."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import AMBIG, TOL, gpu_render, same_ranges

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["fisheye_500k", "lidar_300k", "pinhole_1m"])
def test_fullsize_sampled_parity(name):
    g, s = {"fisheye_500k": lambda: synth.scene_fisheye(0),
            "lidar_300k": lambda: synth.scene_lidar(0),
            "pinhole_1m": lambda: synth.scene_pinhole_large(0)}[name]()
    gp, _ = gpu_render(g, s, moments=True)
    os_ = oracle.OracleSensor(s)
    og = oracle.OracleGaussians(g)
    op = oracle.project(og, os_)
    amb = op["margin"] < AMBIG
    assert np.array_equal(gp["key"], op["key"])
    assert np.array_equal(gp["count"][~amb], op["count"][~amb])
    vis = (~amb) & (op["count"] > 0)
    assert np.array_equal(gp["rect"][:, vis], op["rect"][:, vis])
    # sort order: the oracle bins the GPU's projection -> identical lists and ranges
    ol_g = oracle.bin_pairs(os_, gp["rect"], gp["count"], gp["key"])
    assert gp["n_pairs"] == ol_g["n_pairs"]
    assert np.array_equal(gp["gauss"], ol_g["pair_gauss"])
    assert same_ranges(gp["ranges"], ol_g["ranges"])
    ol = oracle.bin_pairs(os_, op["rect"], op["count"], op["key"]) if amb.any() else ol_g
    ids = np.sort(np.random.default_rng(1).choice(os_.n_rays, 4096, replace=False))
    oo = oracle.composite_rays(og, os_, ol, ids)
    keep = oo["margin"] >= AMBIG
    for k in ("feat", "depth", "alpha") + (("drop",) if os_.kind == 2 else ()):
        d = np.abs(np.asarray(gp[k], np.float64)[..., ids] - oo[k])[..., keep]
        print(name, k, "max-abs", d.max())
        assert d.max() <= TOL, (k, d.max())
    assert np.array_equal(gp["n_proc"][ids][keep], oo["n_proc"][keep])
    print(name, "pairs", gp["n_pairs"], "ambiguous particles", int(amb.sum()), "excluded rays", int((~keep).sum()))
