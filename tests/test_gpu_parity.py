"""Parity of the HIP path (through the C-ABI) with the FP64 oracle on seeded scenes that span
several tiles and ragged tails, plus edge cases, determinism and permutation invariance."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import AMBIG, TOL, d2_representation_error, full_parity, gpu_render, rec_B, to_np

pytestmark = pytest.mark.gpu


def _scene(name):
    if name == "pinhole_128x96":                       # 1,000 particles, 8x6 full tiles
        return synth.scene_pinhole_small(0)
    if name == "pinhole_ragged":                       # 7x5 tiles with partial last row/column
        return synth.scene_pinhole_small(1, n=1500, width=100, height=70, f=80.0)
    if name == "pinhole_sh3_posed":                    # SH degree 3, off-origin rotated camera
        rng = np.random.default_rng(2)
        R_sw = synth.yaw_camera_pose(0.8)
        o = np.array([1.5, -0.7, 0.4], np.float32)
        mean = o[:, None] + R_sw.T.astype(np.float64) @ np.stack(
            [rng.uniform(-3, 3, 3000), rng.uniform(-2, 2, 3000), rng.uniform(1, 12, 3000)])
        g = synth.particles(rng, mean, 0.02, 0.8, 3, synth.FEAT_CAMERA)
        return g, synth.pinhole(120, 88, 90.0, 95.0, cx=61.3, cy=43.9, R_sw=R_sw, origin=o)
    if name == "fisheye_small":
        g, s = synth.scene_fisheye(3, n=20000, width=208, height=136)
        g["mean"] *= np.float32(0.25)
        return g, s
    if name == "lidar_small":
        g, s = synth.scene_lidar(4, n=20000, n_beams=32, n_az=512, n_phi=8, max_per_tile=32)
        g["mean"] *= np.float32(0.2)
        return g, s
    if name == "lidar_nocull":
        g, s = synth.scene_lidar(4, n=20000, n_beams=32, n_az=512, n_phi=8, max_per_tile=32, cull=False)
        g["mean"] *= np.float32(0.2)
        return g, s
    if name == "lidar_posed_m64":
        rng = np.random.default_rng(5)
        n = 15000
        r = rng.uniform(1, 40, n)
        ph = rng.uniform(0, 2 * np.pi, n)
        o = np.array([2.0, -1.0, 0.3], np.float32)
        mean = np.stack([r * np.cos(ph), r * np.sin(ph), rng.uniform(-3, 6, n)]) + o[:, None]
        g = synth.particles(rng, mean, 0.02, 0.6, 0, synth.FEAT_LIDAR)
        g["feat"] = synth.lidar_feat(rng, n)
        s = synth.lidar(synth.beams_uniform(rng, 48), 600, R_sw=synth.yaw_lidar_pose(2.1), origin=o,
                        n_phi=6, max_per_tile=64)
        return g, s
    if name in ("lidar_m128", "lidar_m256", "lidar_m512"):   # large LiDAR tiles (128 / 256 / 512 rays)
        M = int(name[7:])
        g, s = synth.scene_lidar(7, n=20000, n_beams=32, n_az=512, n_phi=4, max_per_tile=M)
        g["mean"] *= np.float32(0.2)
        return g, s
    if name == "pinhole_rolling_shutter":              # camera translating and yawing during readout
        g, s = _scene("pinhole_sh3_posed")
        R1 = synth.yaw_camera_pose(0.92)
        return g, synth.rolling_shutter(s, R1, s["origin"] + np.array([0.6, -0.3, 0.1], np.float32))
    if name == "fisheye_rolling_shutter":
        g, s = _scene("fisheye_small")
        R1 = synth.yaw_camera_pose(0.12)
        return g, synth.rolling_shutter(s, R1, s["origin"] + np.array([0.4, 0.0, 0.2], np.float32))
    if name == "lidar_moving":                         # spinning LiDAR on a moving, turning vehicle
        g, s = _scene("lidar_posed_m64")
        R1 = synth.yaw_lidar_pose(2.25)
        return g, synth.spinning(s, R1, s["origin"] + np.array([1.5, 0.4, 0.0], np.float32))
    if name == "lidar_divergence":                     # beams with a 6 mrad divergence cone
        g, s = _scene("lidar_posed_m64")
        s["beam_divergence"] = 0.006
        return g, s
    if name == "lidar_moving_divergence":
        g, s = _scene("lidar_moving")
        s["beam_divergence"] = 0.02
        return g, s
    if name == "pinhole_wide_aniso":                   # wide field of view, needle/disc particles
        rng = np.random.default_rng(6)                 # (1:1000 axis ratios) close to the camera
        n = 6000
        mean = np.stack([rng.uniform(-6, 6, n), rng.uniform(-4, 4, n), rng.uniform(0.3, 8, n)])
        g = synth.particles(rng, mean, 0.002, 2.0, 0, synth.FEAT_CAMERA)
        return g, synth.pinhole(160, 120, 55.0, 55.0)
    if name in ("pinhole_thin_discs", "pinhole_thin_discs_rs"):
        # discs 1e-3 to 1e-5 as thick as they are wide, 15-60 m away: v^T B v reaches ~1e14,
        # where the difference form of D^2 loses whole units to cancellation
        rng = np.random.default_rng(8)
        n = 4000
        mean = np.stack([rng.uniform(-10, 10, n), rng.uniform(-7, 7, n), rng.uniform(15, 60, n)])
        g = synth.particles(rng, mean, 0.3, 1.5, 0, synth.FEAT_CAMERA)
        w = rng.uniform(np.log(0.3), np.log(1.5), n)
        g["log_scale"] = np.stack([w, w + rng.uniform(-0.5, 0.5, n),
                                   w + rng.uniform(np.log(1e-5), np.log(1e-3), n)]).astype(np.float32)
        s = synth.pinhole(160, 120, 220.0, 220.0)
        if name.endswith("_rs"):
            c, sn = np.cos(0.02), np.sin(0.02)
            R1 = np.array([[c, 0, -sn], [0, 1, 0], [sn, 0, c]], np.float32)
            s = synth.rolling_shutter(s, R1, np.array([0.3, 0.1, 0.2], np.float32))
        return g, s
    if name == "lidar_thin_discs":                     # thin discs around a LiDAR (walls, markings)
        rng = np.random.default_rng(9)
        n = 6000
        r = rng.uniform(8, 45, n)
        ph = rng.uniform(0, 2 * np.pi, n)
        mean = np.stack([r * np.cos(ph), r * np.sin(ph), rng.uniform(-3, 4, n)])
        g = synth.particles(rng, mean, 0.3, 1.2, 0, synth.FEAT_LIDAR)
        g["feat"] = synth.lidar_feat(rng, n)
        w = rng.uniform(np.log(0.3), np.log(1.2), n)
        g["log_scale"] = np.stack([w, w + rng.uniform(-0.5, 0.5, n),
                                   w + rng.uniform(np.log(1e-5), np.log(1e-3), n)]).astype(np.float32)
        return g, synth.lidar(synth.beams_uniform(rng, 32), 512, n_phi=8, max_per_tile=32)
    raise KeyError(name)


SCENES = ["pinhole_128x96", "pinhole_ragged", "pinhole_sh3_posed", "pinhole_wide_aniso", "fisheye_small",
          "lidar_small", "lidar_nocull", "lidar_posed_m64", "lidar_m128", "lidar_m256", "lidar_m512",
          "pinhole_rolling_shutter", "fisheye_rolling_shutter", "lidar_moving", "lidar_divergence",
          "lidar_moving_divergence", "pinhole_thin_discs", "pinhole_thin_discs_rs", "lidar_thin_discs"]


@pytest.mark.parametrize("name", SCENES)
def test_render_parity(name):
    g, s = _scene(name)
    # thin-disc scenes: t_final within the bound of B's float64 representation
    errs, n_ex, gp, oo, _ = full_parity(g, s, eps_d2=d2_representation_error(g) if "thin" in name else 0.0)
    print(name, "max-abs", errs, "excluded rays", n_ex, "pairs", gp["n_pairs"])
    assert gp["n_pairs"] > 1000
    assert n_ex <= 0.001 * oo["alpha"].size
    assert (oo["alpha"] > 0).mean() > 0.05


def test_records_match_particle_definition():
    """Record contents: exp(log opacity) = sigmoid(logit); B = Sigma^{-1} with Sigma from
    scipy's rotation; B v, v^T B v and v = mu - o itself."""
    from scipy.spatial.transform import Rotation
    g, s = _scene("pinhole_sh3_posed")
    gp, _ = gpu_render(g, s)
    rec = gp["records"]
    o = s["origin"].astype(np.float64)
    vis = np.nonzero(gp["count"] > 0)[0]          # records exist for particles that reach a tile
    assert len(vis) > 1000
    for i in vis[::37]:
        w, x, y, z = g["quat"][:, i].astype(np.float64)
        R = Rotation.from_quat([x, y, z, w]).as_matrix()
        sc = np.exp(g["log_scale"][:, i].astype(np.float64))
        B = np.linalg.inv(R @ np.diag(sc * sc) @ R.T)
        Bg = rec_B(rec, i)
        np.testing.assert_allclose(Bg, B, rtol=1e-9, atol=1e-9 * np.abs(B).max())
        v = g["mean"][:, i].astype(np.float64) - o
        np.testing.assert_allclose(rec["bv"][i], B @ v, rtol=1e-9, atol=1e-9 * np.abs(B @ v).max())
        np.testing.assert_allclose(rec["vbv"][i], v @ B @ v, rtol=1e-9)
        np.testing.assert_array_equal(rec["v"][i], v)
        np.testing.assert_allclose(np.exp(rec["log_sigma"][i]), 1 / (1 + np.exp(-np.float64(g["opacity_logit"][i]))),
                                   rtol=1e-14)


def test_determinism_and_permutation_invariance():
    g, s = _scene("pinhole_ragged")
    a, _ = gpu_render(g, s)
    b, _ = gpu_render(g, s)
    for k in ("feat", "depth", "alpha", "t_final", "n_proc", "gauss", "ranges"):
        assert np.array_equal(a[k], b[k]), k
    assert len(np.unique(a["key"])) == len(a["key"])          # tie-free keys
    perm = np.random.default_rng(9).permutation(g["mean"].shape[1])
    c, _ = gpu_render(synth.permute(g, perm), s)
    for k in ("feat", "depth", "alpha", "t_final", "n_proc"):
        assert np.array_equal(a[k], c[k]), k
    assert np.array_equal(perm[c["gauss"]], a["gauss"])


def test_empty_and_fully_culled_scenes():
    g, s = synth.scene_pinhole_small(0, n=50)
    g0 = synth.subset(g, np.arange(0))
    gp, _ = gpu_render(g0, s)
    assert gp["n_pairs"] == 0 and np.all(gp["alpha"] == 0) and np.all(gp["feat"] == 0)
    assert np.all(gp["n_proc"] == 0) and np.all(gp["t_final"] == 1)
    gb = dict(g)
    gb["mean"] = g["mean"].copy()
    gb["mean"][2] *= -1                                         # every particle behind the camera
    gp, _ = gpu_render(gb, s)
    assert gp["n_pairs"] == 0 and int(gp["n_culled"][0]) == 50 and np.all(gp["alpha"] == 0)


def test_degenerate_particles_are_culled_and_counted():
    g, s = synth.scene_pinhole_small(6, n=400)
    g = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    g["mean"][0, 3] = np.nan
    g["quat"][:, 7] = 0.0
    g["log_scale"][1, 11] = np.inf
    g["opacity_logit"][13] = np.nan
    g["mean"][:, 17] = [0.0, 0.0, 0.05]                        # encloses / touches the sensor
    errs, n_ex, gp, oo, _ = full_parity(g, s)
    for i in (3, 7, 11, 13, 17):
        assert gp["count"][i] == 0
    assert int(gp["n_culled"][0]) >= 5


def test_lidar_azimuth_wrap():
    """Particles straddling azimuth 0 get wrapped rects and match the oracle."""
    rng = np.random.default_rng(12)
    n = 3000
    ph = rng.normal(0.0, 0.05, n)
    r = rng.uniform(2, 20, n)
    mean = np.stack([r * np.cos(ph), r * np.sin(ph), rng.uniform(-1, 1, n)])
    g = synth.particles(rng, mean, 0.05, 0.5, 0, synth.FEAT_LIDAR)
    g["feat"] = synth.lidar_feat(rng, n)
    s = synth.lidar(synth.beams_uniform(rng, 32, -10, 10), 512, n_phi=4, max_per_tile=32)
    errs, n_ex, gp, oo, _ = full_parity(g, s)
    ntheta = oracle.OracleSensor(s).c.n_theta
    wrapped = gp["rect"][2] >= ntheta
    assert wrapped.sum() > 50


def test_fisheye_rays_beyond_fov_are_empty():
    g, s = _scene("fisheye_small")
    gp, _ = gpu_render(g, s)
    invalid = ~np.any(s["ray_dir"] != 0, axis=0)
    assert invalid.sum() > 0
    assert np.all(gp["alpha"][invalid] == 0) and np.all(gp["n_proc"][invalid] == 0)


def test_culling_only_removes_particles_without_rays():
    """Culling on vs off (same sensor): the culled particles have no ray in their extent, and
    both renders match their oracle counterparts (Table 7 analogue, correctness side)."""
    g, s_on = _scene("lidar_small")
    _, s_off = _scene("lidar_nocull")
    on, _ = gpu_render(g, s_on)
    off, _ = gpu_render(g, s_off)
    culled = (on["count"] == 0) & (off["count"] > 0)
    assert culled.sum() > 0 and int(on["n_culled"][1]) == culled.sum()
    assert on["n_pairs"] < off["n_pairs"]
    d = np.abs(on["alpha"] - off["alpha"])
    assert np.mean(d == 0) > 0.99


def test_work_counters_leave_outputs_unchanged():
    """The counting variant of the compositing (n_visit, n_pass) writes the same outputs bit for
    bit, and its counters are ordered: entries passing the pre-test <= entries evaluated <= list
    positions visited (n_proc)."""
    import torch
    import paper_2510_12901_amd as ut
    g_np, s_np = _scene("pinhole_sh3_posed")
    g = ut.GaussianSet.from_numpy(g_np)
    s = ut.Sensor(s_np)
    p, bins, a = ut.render(g, s, state=True)
    b = ut.alloc_out(s, g.mean.device, state=True, counters=True)
    ut.composite(p, bins, s, out=b)
    torch.cuda.synchronize()
    for k in ("feat", "depth", "alpha", "t_final", "n_proc"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    nproc, nvis, npass = (to_np(t).view(np.uint32).astype(np.int64) for t in (b.n_proc, b.n_visit, b.n_pass))
    assert np.all(npass <= nvis) and np.all(nvis <= nproc)
    assert nvis.sum() < nproc.sum() and npass.sum() > 0


def test_large_lidar_tiles_rejected_by_batch_and_adjoint():
    """Tiles of more than 256 rays render on the plain path only; the batched composite and
    the adjoint refuse them with UT_ERR_UNSUPPORTED instead of dropping rays."""
    import paper_2510_12901_amd as ut
    from paper_2510_12901_amd import _abi as A
    g_np, s_np = _scene("lidar_m512")
    g = ut.GaussianSet.from_numpy(g_np)
    s = ut.Sensor(s_np)
    assert s.max_tile_rays > 256
    p, bins, out = ut.render(g, s)
    with pytest.raises(A.UtError, match="unsupported"):
        ut.composite_batch([(p, bins, s, out)])


@pytest.mark.parametrize("n_workgroups", [1024, 0])
def test_batched_composite_with_moving_and_static_sensors(n_workgroups):
    """The batched composite (persistent workgroups, or one workgroup per item) handles a
    moving sensor's per-ray origins and LiDAR units: every output is bit-identical to the
    plain single-request call."""
    import torch
    import paper_2510_12901_amd as ut
    items, plain = [], []
    for name in ("pinhole_rolling_shutter", "pinhole_ragged", "lidar_moving", "lidar_small"):
        g_np, s_np = _scene(name)
        g = ut.GaussianSet.from_numpy(g_np)
        s = ut.Sensor(s_np)
        p, bins, a = ut.render(g, s, state=True)
        b = ut.alloc_out(s, g.mean.device, state=True)
        items.append((p, bins, s, b))
        plain.append(a)
    ut.composite_batch(items, n_workgroups=n_workgroups)
    torch.cuda.synchronize()
    for (p, bins, s, b), a in zip(items, plain):
        for k in ("feat", "depth", "alpha", "t_final", "n_proc"):
            assert torch.equal(getattr(a, k), getattr(b, k)), k


def test_beam_divergence_records():
    """With beam divergence the record's quadric is B = Sigma_hat^{-1} for
    Sigma_hat = Sigma + (r tan(theta/2))^2 (I - d d^T) (built here with scipy's rotation)."""
    from scipy.spatial.transform import Rotation
    g_np, s_np = _scene("lidar_divergence")
    gp, _ = gpu_render(g_np, s_np)
    rec = gp["records"]
    o = s_np["origin"].astype(np.float64)
    vis = np.nonzero(gp["count"] > 0)[0]
    assert len(vis) > 1000
    for i in vis[::41]:
        w, x, y, z = g_np["quat"][:, i].astype(np.float64)
        R = Rotation.from_quat([x, y, z, w]).as_matrix()
        sc = np.exp(g_np["log_scale"][:, i].astype(np.float64))
        v = g_np["mean"][:, i].astype(np.float64) - o
        r = np.linalg.norm(v)
        d = v / r
        S_hat = R @ np.diag(sc * sc) @ R.T + (r * np.tan(0.003)) ** 2 * (np.eye(3) - np.outer(d, d))
        B = np.linalg.inv(S_hat)
        np.testing.assert_allclose(rec_B(rec, i), B, rtol=1e-8, atol=1e-8 * np.abs(B).max())
        np.testing.assert_allclose(rec["bv"][i], B @ v, rtol=1e-8, atol=1e-8 * np.abs(B @ v).max())
        np.testing.assert_allclose(rec["vbv"][i], v @ B @ v, rtol=1e-8)


@pytest.mark.parametrize("abk", [(1.0, 2.0, 0.0), (1.0, 0.0, 1.0)])
def test_offscreen_precull_matches_full_projection(abk):
    """Without moments the static pinhole projection skips the UT of particles whose 3-sigma
    rect certainly misses the image; every output must equal the full path (moments
    requested), on a scene with particles all around a posed camera, some huge, some at the
    image border."""
    import torch
    import paper_2510_12901_amd as ut
    rng = np.random.default_rng(21)
    n = 60000
    mean = np.stack([rng.uniform(-30, 30, n), rng.uniform(-30, 30, n), rng.uniform(-4, 4, n)])
    g_np = synth.particles(rng, mean, 0.01, 3.0, 3, synth.FEAT_CAMERA)
    s_np = synth.pinhole(200, 150, 160.0, 150.0, cx=97.0, cy=71.0, R_sw=synth.yaw_camera_pose(0.7),
                         origin=np.array([0.5, -1.0, 0.2], np.float32))
    g = ut.GaussianSet.from_numpy(g_np)
    s = ut.Sensor(s_np)
    full = ut.project(g, s, abk=abk, moments=True)
    fast = ut.project(g, s, abk=abk, moments=False)
    torch.cuda.synchronize()
    for k in ("rect", "key", "count", "trect", "n_culled"):
        assert torch.equal(getattr(full, k), getattr(fast, k)), k
    vis = torch.nonzero(full.count > 0).flatten()
    from paper_2510_12901_amd import _abi as A
    rb = A.RECORD_BYTES
    fr = full.records.view(-1, rb)[vis]
    qr = fast.records.view(-1, rb)[vis]
    assert torch.equal(fr, qr)
    # the scene exercises the skip: many particles lie well in front of the camera yet project
    # far outside the image
    v = np.asarray(s_np["R_sw"], np.float64) @ (mean - np.asarray(s_np["origin"], np.float64)[:, None])
    u = 160.0 * v[0] / v[2] + 97.0
    far_off = (v[2] > 2.0) & ((u < -150) | (u > 350))
    assert far_off.sum() > n // 10


@pytest.mark.parametrize("name", ["lidar_small", "lidar_posed_m64", "lidar_m128", "lidar_m256"])
def test_lidar_compositing_units_partition_the_tiles(name):
    """The compositing units built at sensor set-up: every azimuth-elevation tile lies in
    exactly one unit; a unit is a run of at most 4 adjacent tiles of one elevation tile inside
    one super-tile column; its rays fit unit_rays lanes, the smallest of 64, 128, 256 that
    holds the largest tile (and 256 lanes in the batched kernel's packing)."""
    import paper_2510_12901_amd as ut
    g_np, s_np = _scene(name)
    s = ut.Sensor(s_np)
    c = s.c
    NP, NT = c.n_phi, c.n_theta
    al = lambda v: (v + 255) // 256 * 256
    cull = (c.cull_az + 1) * (c.cull_el + 1) if c.cull else 1
    off = al(8 * (NP + 1)) + al(4 * (NP + 1)) + al(4 * cull)
    tb = to_np(s.tables)
    units = tb[off: off + 16 * c.n_units].view(np.int32).reshape(-1, 4)
    bstart = tb[al(8 * (NP + 1)): al(8 * (NP + 1)) + 4 * (NP + 1)].view(np.int32)
    assert c.unit_rays == min(u for u in (64, 128, 256) if u >= s.max_tile_rays)
    wide = tb[off + 16 * NP * NT: off + 16 * NP * NT + 16 * c.n_units_wide].view(np.int32).reshape(-1, 4)
    assert 0 < c.n_units_wide <= c.n_units
    az0 = lambda j: (j * c.n_az + NT - 1) // NT
    for table, cap in ((units, c.unit_rays), (wide, 256)):   # single-request and batched packings
        seen = np.zeros((NP, NT), np.int64)
        for k, j0, j1, rays in table:
            assert 0 <= k < NP and 0 <= j0 < j1 <= NT and j1 - j0 <= 4
            assert j0 // 8 == (j1 - 1) // 8
            assert rays == (bstart[k + 1] - bstart[k]) * (az0(j1) - az0(j0)) <= cap
            seen[k, j0:j1] += 1
        assert np.all(seen == 1)


@pytest.mark.parametrize("name", ["lidar_small", "lidar_posed_m64", "lidar_m128", "lidar_m256", "lidar_moving",
                                  "lidar_divergence", "lidar_thin_discs"])
def test_lidar_units_match_the_per_tile_kernel(name):
    """The unit kernel (several azimuth tiles per workgroup, one list per tile built in LDS)
    against the one-tile-per-workgroup kernel on the same projection and bins: every ray
    walks the same list in the same order, so the per-ray outputs, the processed counts and
    the per-tile bin ends agree exactly."""
    import torch
    import paper_2510_12901_amd as ut
    g_np, s_np = _scene(name)
    S = ut.Sensor(s_np)
    assert S.c.n_units > 0 and S.c.unit_rays > 0
    p = ut.project(ut.GaussianSet.from_numpy(g_np), S)
    bins = ut.bin_and_sort(p, S)
    unit = ut.composite(p, bins, S)
    n_units = S.c.n_units
    S.c.n_units = 0                      # dispatch falls back to one tile per workgroup
    try:
        tile = ut.composite(p, bins, S)
    finally:
        S.c.n_units = n_units
    torch.cuda.synchronize()
    for f in ("n_proc", "tile_end"):
        assert torch.equal(getattr(unit, f), getattr(tile, f)), f
    assert int(unit.n_proc.max().item()) > 0
    for f in ("feat", "depth", "alpha", "drop", "t_final"):
        a, b = getattr(unit, f), getattr(tile, f)
        d = float((a.double() - b.double()).abs().max().item())
        print(name, f, "max |unit - tile|", d)
        assert d == 0.0, f
