"""Spatial order of a resident particle set (ut_spatial_order, ut_gather_gaussians): the
permutation follows the Morton code defined in utrast.h, and a reordered set renders and
differentiates the same as the original."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import to_np
from test_gpu_parity import _scene

pytestmark = pytest.mark.gpu


def _morton_np(mean):
    """30-bit Morton codes by the header's definition, float32 arithmetic like the kernel."""
    m = np.asarray(mean, np.float32)
    fin = np.all(np.isfinite(m), axis=0)
    lo = m[:, fin].min(axis=1)
    hi = m[:, fin].max(axis=1)
    ext = (hi - lo).astype(np.float32)
    q = np.zeros((3, m.shape[1]), np.uint64)
    for c in range(3):
        with np.errstate(invalid="ignore"):
            f = ((m[c] - lo[c]) / ext[c]).astype(np.float32) if ext[c] > 0 else np.zeros(m.shape[1], np.float32)
            v = np.minimum(np.maximum(f * np.float32(1023.0), np.float32(0.0)), np.float32(1023.0))
        q[c] = np.where(fin, v, 0).astype(np.uint64)

    def spread(x):
        x = (x | (x << np.uint64(16))) & np.uint64(0x030000FF)
        x = (x | (x << np.uint64(8))) & np.uint64(0x0300F00F)
        x = (x | (x << np.uint64(4))) & np.uint64(0x030C30C3)
        return (x | (x << np.uint64(2))) & np.uint64(0x09249249)
    code = spread(q[0]) | (spread(q[1]) << np.uint64(1)) | (spread(q[2]) << np.uint64(2))
    return np.where(fin, code, np.uint64(0xFFFFFFFF))


def test_spatial_order_is_the_morton_permutation():
    import paper_2510_12901_amd as ut
    rng = np.random.default_rng(3)
    n = 70000
    mean = np.stack([rng.uniform(-50, 50, n), rng.uniform(-5, 5, n), rng.uniform(-50, 50, n)])
    g_np = synth.particles(rng, mean, 0.02, 1.0, 1, synth.FEAT_CAMERA)
    g_np["mean"][:, [5, 77, 4000]] = np.float32(np.nan)   # non-finite means go last
    g = ut.GaussianSet.from_numpy(g_np)
    perm = to_np(ut.spatial_order(g)).astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(n))
    want = np.argsort(_morton_np(g_np["mean"]), kind="stable")
    assert np.array_equal(perm, want)
    assert set(perm[-3:].tolist()) == {5, 77, 4000}
    r = ut.gather(g, torch.as_tensor(perm.astype(np.int32), device="cuda"))
    for k in ("mean", "quat", "log_scale", "opacity_logit", "feat"):
        a, b = to_np(getattr(g, k)), to_np(getattr(r, k))
        assert np.array_equal(b, a[..., perm], equal_nan=True), k


@pytest.mark.parametrize("name", ["pinhole_sh3_posed", "lidar_posed_m64"])
def test_reordered_set_renders_and_differentiates_the_same(name):
    import paper_2510_12901_amd as ut
    g_np, s_np = _scene(name)
    g = ut.GaussianSet.from_numpy(g_np)
    s = ut.Sensor(s_np)
    perm = ut.spatial_order(g)
    r = ut.gather(g, perm)
    p0, b0, o0 = ut.render(g, s)
    p1, b1, o1 = ut.render(r, s)
    torch.cuda.synchronize()
    for k in ("feat", "depth", "alpha", "n_proc", "t_final"):
        assert torch.equal(getattr(o0, k), getattr(o1, k)), k
    up = torch.as_tensor(np.random.default_rng(1).standard_normal((3, s.n_rays)).astype(np.float32), device="cuda")
    g0 = ut.backward(g, p0, b0, s, o0, up_feat=up)
    g1 = ut.backward(r, p1, b1, s, o1, up_feat=up)
    torch.cuda.synchronize()
    pn = to_np(perm).astype(np.int64)
    for k in ("mean", "quat", "log_scale", "opacity_logit", "feat"):
        a, b = to_np(g0[k]).astype(np.float64)[..., pn], to_np(g1[k]).astype(np.float64)
        scale = np.abs(a).max() + 1e-30
        assert np.abs(a - b).max() <= 1e-5 * scale, k
