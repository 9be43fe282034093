"""ut_composite_batch_noalloc (the batched composite on the library's fixed per-GPU queue)
gives exactly the outputs of ut_composite_batch with a caller workspace, on two calls in a
row (the second with fewer, smaller requests), and refuses more items than its queue holds."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

KEYS = ("feat", "depth", "alpha")


def _requests(specs):
    import torch
    import paper_2510_12901_amd as ut
    reqs = []
    for g_np, s_np in specs:
        g = ut.GaussianSet.from_numpy(g_np)
        s = ut.Sensor(s_np)
        p = ut.project(g, s)
        bins = ut.bin_and_sort(p, s)
        reqs.append((p, bins, s))
    torch.cuda.synchronize()
    return reqs


def _outs(reqs, fill):
    import paper_2510_12901_amd as ut
    outs = []
    for p, bins, s in reqs:
        o = ut.alloc_out(s, p.records.device, state=False)
        for k in KEYS + (("drop",) if s.is_lidar else ()):
            getattr(o, k).fill_(fill)      # stale values must be overwritten
        outs.append(o)
    return outs


def _check_same(reqs, a, b):
    for (p, bins, s), oa, ob in zip(reqs, a, b):
        for k in KEYS + (("drop",) if s.is_lidar else ()):
            assert getattr(oa, k).numel() == s.n_rays * (3 if k == "feat" else 1)
            assert np.isfinite(getattr(ob, k).cpu().numpy()).all(), k
            assert np.array_equal(getattr(oa, k).cpu().numpy(), getattr(ob, k).cpu().numpy()), k


def test_noalloc_batch_matches_workspace_batch_twice():
    import torch
    import paper_2510_12901_amd as ut

    first = [synth.scene_pinhole_small(0),
             synth.scene_pinhole_small(1, n=1500, width=100, height=70, f=80.0),
             synth.scene_lidar(4, n=20000, n_beams=32, n_az=512, n_phi=8, max_per_tile=32)]
    g, s = synth.scene_pinhole_small(3, n=1200, width=120, height=88, f=90.0)
    cam_mv = synth.rolling_shutter(s, synth.yaw_camera_pose(0.1), s["origin"] + np.array([0.3, 0.0, 0.0], np.float32))
    first.append((g, cam_mv))
    second = [synth.scene_pinhole_small(5, n=400, width=40, height=30, f=30.0)]

    for specs in (first, second):     # second call: fewer items, fewer tiles, fewer rays
        reqs = _requests(specs)
        ref = _outs(reqs, -1.0)
        ut.composite_batch([(p, b, s, o) for (p, b, s), o in zip(reqs, ref)])
        got = _outs(reqs, float("nan"))
        ut.composite_batch_noalloc([(p, b, s, o) for (p, b, s), o in zip(reqs, got)])
        torch.cuda.synchronize()
        _check_same(reqs, ref, got)
        # the plain single-request path agrees too
        for (p, bins, s), o in zip(reqs, got):
            a = ut.composite(p, bins, s, state=False)
            torch.cuda.synchronize()
            for k in KEYS:
                assert torch.equal(getattr(a, k), getattr(o, k)), k


def test_noalloc_batch_rejects_more_items_than_its_queue():
    from paper_2510_12901_amd import _abi as A
    L = A.lib()
    n = A.BATCH_NOALLOC_MAX_ITEMS + 1
    arr = (A.UtBatchItem * n)()
    prm = A.UtRenderParams(1 / 255, 0.99, 1e-4)
    assert L.ut_composite_batch_noalloc(C.cast(arr, C.c_void_p), n, A.ref(prm), 64, None) == A.UT_ERR_CAPACITY
    assert L.ut_composite_batch_noalloc(None, 1, A.ref(prm), 64, None) == A.UT_ERR_ARG
