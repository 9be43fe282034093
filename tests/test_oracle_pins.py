"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
closed forms, library routines, brute force, hand-worked fixtures and invariants.
CPU only."""
import json
import os

import numpy as np
import pytest
from scipy.optimize import minimize_scalar
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sigma_from_params(g, i):
    """Covariance from scipy's quaternion->rotation (scalar-last order)."""
    w, x, y, z = g["quat"][:, i].astype(np.float64)
    R = Rotation.from_quat([x, y, z, w]).as_matrix()
    s = np.exp(g["log_scale"][:, i].astype(np.float64))
    return R @ np.diag(s * s) @ R.T


def _one(g, i):
    return synth.subset(g, [i])


# ------------------------------------------------------------------ unscented transform
@pytest.mark.parametrize("abk", [(1.0, 2.0, 0.0), (0.5, 2.0, 1.0), (1.3, 0.0, 2.0)])
def test_ut_exact_for_linear_projection(abk):
    """Sec. 3.2 UT: for an affine sensor map the 7-point UT reproduces A mu + b and A Sigma A^T."""
    rng = np.random.default_rng(11)
    yaw = 0.7
    R_sw = synth.yaw_camera_pose(yaw)
    origin = np.array([0.3, -0.2, 0.5], np.float32)
    s = synth.pinhole(64, 48, 3.0, 2.5, cx=31.0, cy=22.0, R_sw=R_sw, origin=origin, kind=synth.ORTHO)
    n = 200
    mean = np.stack([rng.uniform(-5, 5, n), rng.uniform(-5, 5, n), rng.uniform(-1, 1, n)])
    fwd = R_sw[2].astype(np.float64)
    mean = mean + 20.0 * fwd[:, None]            # in front of the sensor
    g = synth.particles(rng, mean, 0.05, 2.0, 0, synth.FEAT_CAMERA)
    proj = oracle.project(g, s, abk)
    assert proj["valid"].all()
    A = np.diag([3.0, 2.5]) @ R_sw[:2].astype(np.float64)
    for i in range(n):
        mu = g["mean"][:, i].astype(np.float64)
        m_ref = A @ (mu - origin.astype(np.float64)) + np.array([31.0, 22.0])
        S = A @ _sigma_from_params(g, i) @ A.T
        np.testing.assert_allclose(proj["mean2"][:, i], m_ref, rtol=0, atol=1e-12)
        np.testing.assert_allclose(proj["cov2"][:, i], [S[0, 0], S[0, 1], S[1, 1]], rtol=1e-11, atol=1e-12)


def test_ut_close_to_monte_carlo_pinhole():
    """App. (LiDAR projection, Table 8): UT moments are close to Monte Carlo moments for
    small particles (statistical; 4x10^5 samples)."""
    rng = np.random.default_rng(3)
    g, s = synth.scene_pinhole_small(5, n=20)
    proj = oracle.project(g, s)
    for i in range(5):
        S = _sigma_from_params(g, i)
        x = rng.multivariate_normal(g["mean"][:, i].astype(np.float64), S, 400000)
        u = 100.0 * x[:, 0] / x[:, 2] + 64.0
        v = 100.0 * x[:, 1] / x[:, 2] + 48.0
        mc_m = np.array([u.mean(), v.mean()])
        mc_c = np.cov(np.stack([u, v]))
        scale = np.sqrt(mc_c[0, 0] + mc_c[1, 1])
        assert np.all(np.abs(proj["mean2"][:, i] - mc_m) < 0.05 * scale)
        np.testing.assert_allclose([proj["cov2"][0, i], proj["cov2"][2, i]], [mc_c[0, 0], mc_c[1, 1]], rtol=0.05)


# Nonlinear sensor maps.  A particle stretched along one axis only (the other two scales
# 1e-5 of it) makes the projection a function of one Gaussian scalar t ~ N(0, s^2); the
# exact moments of that function follow from the Gaussian's moments E[t^2k] = (2k-1)!! s^2k,
# expanded in s.  The 7-point UT, whose axis points sit at mu +- sqrt(c) L_i with
# c = alpha^2 (3 + kappa), reproduces the Gaussian's moments up to the fourth only when
# c = 3, so its mean and variance agree with the exact ones through s^4 there and differ at
# s^4 by terms that depend on (alpha, beta, kappa) otherwise.  Each check compares the
# normalised s^4 coefficient, (value - lower orders) / s^4, at s = 0.005 (s^6 terms < 0.02).
def _stretched(mean, axis, sigma):
    rng = np.random.default_rng(0)
    g = synth.particles(rng, np.asarray(mean, np.float64).reshape(3, 1), 1.0, 1.0, 0, synth.FEAT_CAMERA)
    g["quat"] = np.array([[1.0], [0.0], [0.0], [0.0]], np.float32)
    ls = np.full((3, 1), np.log(1e-5 * sigma), np.float32)
    ls[axis, 0] = np.log(sigma)
    g["log_scale"] = ls
    return g, float(np.exp(np.float64(ls[axis, 0])))


@pytest.mark.parametrize("abk", [(1.0, 0.0, 0.0), (1.0, 2.0, 0.0), (0.5, 2.0, 1.0), (1.3, 0.0, 2.0)])
def test_ut_pinhole_depth_stretched_series(abk):
    """Sec. 3.2 UT through the pinhole map.  A particle at (x0, y0, z0) stretched along the
    optical axis projects to u - cx = f x0 / z, v - cy = f y0 / z with z = z0 (1 + t).
    Exact Gaussian moments: E[1/(1+t)] = 1 + s^2 + 3 s^4, Var[1/(1+t)] = s^2 + 8 s^4 (+O(s^6)).
    The UT gives 1 + s^2 + c s^4 and s^2 + (3c - alpha^2 + beta) s^4 (expansion of its seven
    points: four collapse onto the mean, two sit at z0 (1 +- sqrt(c) s)); with
    (alpha, beta, kappa) = (1, 0, 0) both equal the exact moments, and beta enters the
    variance only through the centre point, one-for-one."""
    a, b, k = abk
    c = a * a * (3.0 + k)
    s_cam = synth.pinhole(64, 48, 90.0, 80.0, cx=30.0, cy=20.0)
    for z0 in (8.0, 20.0):
        g, sigma = _stretched([0.6 * z0, -0.4 * z0, z0], 2, 0.005 * z0)
        x0, y0, zz = (float(v) for v in g["mean"][:, 0].astype(np.float64))
        s = sigma / zz
        pr = oracle.project(g, s_cam, abk)
        assert pr["valid"][0]
        mu = (pr["mean2"][0, 0] - 30.0) / (90.0 * x0 / zz)
        mv = (pr["mean2"][1, 0] - 20.0) / (80.0 * y0 / zz)
        for m in (mu, mv):
            assert abs((m - 1.0 - s * s) / s**4 - c) < 0.005 * c + 0.005
        var = np.array([pr["cov2"][0, 0] / (90.0 * x0 / zz) ** 2,
                        pr["cov2"][1, 0] / (90.0 * 80.0 * x0 * y0 / zz**2),
                        pr["cov2"][2, 0] / (80.0 * y0 / zz) ** 2])
        c4 = (var - s * s) / s**4
        np.testing.assert_allclose(c4, 3 * c - a * a + b, atol=0.01 + 0.002 * (3 * c))
        if abk == (1.0, 0.0, 0.0):
            np.testing.assert_allclose(c4, 8.0, atol=0.01)      # exact Var[1/(1+t)]


@pytest.mark.parametrize("where, axis", [((0.0, 1.0, 0.0), 0), ((0.0, 1.0, 0.0), 2), ((1.0, 0.0, 0.0), 1)])
def test_ut_lidar_angles_stretched_series(where, axis):
    """Eq. 3 map through the UT.  A particle at distance r0 stretched across the line of
    sight moves one angle by atan(t): along the horizontal the azimuth, along z the
    elevation, asin(z / r) = atan(t).  Exact: mean unchanged by symmetry, Var[atan t] =
    s^2 - 2 s^4 + O(s^6); the UT (c = 3) agrees through s^4.  The particle on the +x axis
    has sigma azimuths on both sides of 0 = 2 pi (they must be unwrapped around the mean's)."""
    ls = synth.lidar(np.deg2rad(np.linspace(-20.0, 20.0, 16)), 256)
    r0 = 15.0
    g, sigma = _stretched(r0 * np.array(where), axis, 0.005 * r0)
    s = sigma / r0
    pr = oracle.project(g, ls)
    assert pr["valid"][0]
    moved = 1 if axis == 2 else 0
    centre = np.arctan2(where[1], where[0]) if moved == 0 else 0.0
    d = (pr["mean2"][moved, 0] - centre + np.pi) % (2 * np.pi) - np.pi
    assert abs(d) < 1e-14
    var = pr["cov2"][0 if moved == 0 else 2, 0]
    assert abs((var - s * s) / s**4 - (-2.0)) < 0.01
    # the other angle sees only the 1e-5 side scales: variance ~(1e-5 s)^2, no s^2 term
    assert pr["cov2"][2 if moved == 0 else 0, 0] < 1e-5 * s * s
    assert abs(pr["cov2"][1, 0]) < 1e-5 * s * s


def test_ut_fisheye_axis_stretched_series():
    """Equidistant fisheye through the UT.  A particle on the optical axis at depth z0
    stretched along x maps to u - cx = f d(atan t), d(theta) = theta (1 + k1 theta^2 + ...).
    Exact: mean cx by symmetry, Var = f^2 (s^2 + (6 k1 - 2) s^4 + O(s^6)); the UT agrees
    through s^4."""
    k = [0.04, -0.01, 0.005, 0.0]
    fe = synth.fisheye(96, 64, k)
    f = fe["fx"]
    z0 = 12.0
    g, sigma = _stretched([0.0, 0.0, z0], 0, 0.005 * z0)
    s = sigma / z0
    pr = oracle.project(g, fe)
    assert pr["valid"][0]
    assert abs(pr["mean2"][0, 0] - fe["cx"]) < 1e-12 * f
    var = pr["cov2"][0, 0] / (f * f)
    assert abs((var - s * s) / s**4 - (6 * k[0] - 2.0)) < 0.01


# ------------------------------------------------------------------ projections
def test_projection_round_trip_of_ray_tables():
    """Every camera ray of the generator's table, pushed out to 7 m, projects back to its
    pixel centre (fisheye: Newton-inverted distortion vs the oracle's forward model)."""
    rng = np.random.default_rng(0)
    k = synth.fisheye_distortion(rng, np.deg2rad(95))
    for s in (synth.fisheye(96, 64, k, R_sw=synth.yaw_camera_pose(0.4), origin=[1, 2, 0.5]),
              synth.pinhole(40, 30, 35.0, 33.0, cx=19.5, cy=14.0, R_sw=synth.yaw_camera_pose(2.0), origin=[0, 1, 0])):
        d = s["ray_dir"].astype(np.float64)
        valid = np.any(d != 0, axis=0)
        pts = s["origin"].astype(np.float64)[None] + 7.0 * d.T
        uv, ok = oracle.project_points(s, pts)
        W = s["width"]
        idx = np.arange(d.shape[1])
        centre = np.stack([idx % W + 0.5, idx // W + 0.5], 1)
        assert ok[valid].all()
        assert np.abs(uv[valid] - centre[valid]).max() < 2e-3   # float32 ray rounding
        if s["kind"] == synth.FISHEYE:
            assert (~valid).sum() > 0                            # corners beyond theta_max


def test_lidar_projection_eq3():
    """Eq. 3: ray (b, a) at range 30 m maps to (2 pi a / A, elevation_b)."""
    s = synth.lidar(np.deg2rad([-20.0, -3.0, 0.0, 7.5, 14.0]), 64, R_sw=synth.yaw_lidar_pose(1.1), origin=[3, -2, 1])
    d = s["ray_dir"].astype(np.float64)
    pts = s["origin"].astype(np.float64)[None] + 30.0 * d.T
    uv, ok = oracle.project_points(s, pts)
    assert ok.all()
    a = np.arange(d.shape[1]) % 64
    b = np.arange(d.shape[1]) // 64
    dphi = (uv[:, 0] - 2 * np.pi * a / 64 + np.pi) % (2 * np.pi) - np.pi
    assert np.abs(dphi).max() < 1e-6
    assert np.abs(uv[:, 1] - s["beam_elev"].astype(np.float64)[b]).max() < 1e-6
    # axis points in the sensor frame
    s0 = synth.lidar([0.0, 0.1], 8)
    uv, ok = oracle.project_points(s0, [[5, 0, 0], [0, 5, 0], [-5, 0, 0], [0, -5, 0], [3, 0, 4]])
    np.testing.assert_allclose(uv[:, 0], [0, np.pi / 2, np.pi, 3 * np.pi / 2, 0], atol=1e-15)
    np.testing.assert_allclose(uv[:, 1], [0, 0, 0, 0, np.arcsin(0.8)], atol=1e-15)


# ------------------------------------------------------------------ spherical harmonics
def test_sh_matches_scipy_and_is_orthonormal():
    rng = np.random.default_rng(1)
    d = rng.standard_normal((500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = oracle.sh_eval(3, d)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    for l in range(4):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), theta, phi)      # complex, Condon-Shortley phase
            ref = c.real if m == 0 else (np.sqrt(2) * c.real if m > 0 else np.sqrt(2) * c.imag)
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-12)
    # Gauss-Legendre x uniform-azimuth quadrature: exact for these polynomial degrees
    zt, zw = np.polynomial.legendre.leggauss(12)
    ph = np.arange(24) * 2 * np.pi / 24
    Z, P = np.meshgrid(zt, ph, indexing="ij")
    W = np.repeat(zw, 24) * (2 * np.pi / 24)
    r = np.sqrt(1 - Z.ravel() ** 2)
    dirs = np.stack([r * np.cos(P.ravel()), r * np.sin(P.ravel()), Z.ravel()], 1)
    Yq = oracle.sh_eval(3, dirs)
    G = (Yq * W[:, None]).T @ Yq
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


# ------------------------------------------------------------------ response and compositing
def test_single_isotropic_gaussian_closed_form():
    """Eq. 1 with one particle: C = c alpha, depth = tau* alpha, omega = alpha, with
    tau* = mu.d and D^2 = |mu x d|^2 / s^2 for an isotropic particle and a camera at 0."""
    s = synth.pinhole(64, 64, 60.0, 60.0)
    mu = np.array([[0.15], [-0.1], [3.0]])
    g = synth.particles(np.random.default_rng(0), mu, 0.2, 0.2, 0, synth.FEAT_CAMERA,
                        dc=synth.camera_rgb_dc(np.array([[0.9], [0.4], [0.2]])))
    g["log_scale"][:] = np.float32(np.log(0.2))
    g["opacity_logit"][:] = np.float32(np.log(0.3 / 0.7))
    sigma = 1.0 / (1.0 + np.exp(-np.float64(g["opacity_logit"][0])))
    sc = np.exp(np.float64(g["log_scale"][0, 0]))
    proj, lists, out = oracle.render(g, s)
    d = s["ray_dir"].astype(np.float64).T
    m = mu.ravel().astype(np.float32).astype(np.float64)
    dd = np.sum(d * d, axis=1)                  # float32 rays are unit only to ~1e-7
    tau = d @ m / dd
    D2 = np.sum(np.cross(m, d) ** 2, axis=1) / (sc**2 * dd)
    alpha = np.minimum(sigma * np.exp(-0.5 * D2), 0.99)
    alpha = np.where(alpha < 1 / 255, 0.0, alpha)
    col = g["feat"][0, :, 0].astype(np.float64) / synth.DC_SCALE + 0.5
    assert (alpha > 0).sum() > 100
    np.testing.assert_allclose(out["alpha"], alpha, atol=1e-13)
    np.testing.assert_allclose(out["depth"], tau * alpha, atol=1e-12)
    np.testing.assert_allclose(out["feat"], col[:, None] * alpha[None], atol=1e-13)


def test_two_gaussians_closed_form():
    """C = c1 a1 + c2 a2 (1 - a1), nearer particle first."""
    s = synth.pinhole(32, 32, 30.0, 30.0)
    mu = np.array([[0.05, -0.04], [0.02, 0.03], [2.0, 3.5]])
    g = synth.particles(np.random.default_rng(0), mu, 0.3, 0.3, 0, synth.FEAT_CAMERA,
                        dc=synth.camera_rgb_dc(np.array([[0.9, 0.1], [0.2, 0.8], [0.5, 0.5]])))
    g["log_scale"][:] = np.float32(np.log(0.3))
    g["opacity_logit"][:] = np.float32(np.log(0.25 / 0.75))
    proj, lists, out = oracle.render(g, s)
    d = s["ray_dir"].astype(np.float64).T
    sc = np.exp(np.float64(g["log_scale"][0, 0]))
    sig = 1.0 / (1.0 + np.exp(-np.float64(g["opacity_logit"][0])))
    a, t, c = [], [], []
    dd = np.sum(d * d, axis=1)
    for i in range(2):
        m = g["mean"][:, i].astype(np.float64)
        al = np.minimum(sig * np.exp(-0.5 * np.sum(np.cross(m, d) ** 2, 1) / (sc**2 * dd)), 0.99)
        a.append(np.where(al < 1 / 255, 0, al))
        t.append(d @ m / dd)
        c.append(g["feat"][0, :, i].astype(np.float64) / synth.DC_SCALE + 0.5)
    Cref = c[0][:, None] * a[0] + c[1][:, None] * a[1] * (1 - a[0])
    np.testing.assert_allclose(out["feat"], Cref, atol=1e-13)
    np.testing.assert_allclose(out["depth"], t[0] * a[0] + t[1] * a[1] * (1 - a[0]), atol=1e-12)
    np.testing.assert_allclose(out["t_final"], (1 - a[0]) * (1 - a[1]), atol=1e-14)


def test_response_is_numeric_maximum_along_ray():
    """Sec. 3.2 (3DGRT response): tau* maximises rho along the ray; checked against a 1D
    numeric minimiser of the Mahalanobis distance with scipy's rotation matrices."""
    rng = np.random.default_rng(4)
    s = synth.pinhole(16, 16, 12.0, 12.0, R_sw=synth.yaw_camera_pose(0.3), origin=[0.5, -0.5, 0.2])
    mean = (s["origin"].astype(np.float64)[:, None] + 4.0 * s["R_sw"][2].astype(np.float64)[:, None]
            + rng.uniform(-0.5, 0.5, (3, 6)))
    for i in range(6):
        g = synth.particles(rng, mean[:, i:i + 1], 0.1, 1.2, 0, synth.FEAT_CAMERA,
                            dc=synth.camera_rgb_dc(np.full((3, 1), 0.75)))
        g["opacity_logit"][:] = np.float32(np.log(0.6 / 0.4))
        proj, lists, out = oracle.render(g, s)
        B = np.linalg.inv(_sigma_from_params(g, 0))
        mu = g["mean"][:, 0].astype(np.float64)
        o = s["origin"].astype(np.float64)
        sig = 1.0 / (1.0 + np.exp(-np.float64(g["opacity_logit"][0])))
        for r in rng.choice(256, 40, replace=False):
            if proj["count"][0] == 0:
                break
            d = s["ray_dir"][:, r].astype(np.float64)
            f = lambda t: (o + t * d - mu) @ B @ (o + t * d - mu)
            res = minimize_scalar(f, bounds=(-50.0, 50.0), method="bounded", options={"xatol": 1e-11})
            al = min(sig * np.exp(-0.5 * res.fun), 0.99)
            tx, ty = (r % 16) // 16, (r // 16) // 16
            if al < 1 / 255:
                assert out["alpha"][r] == 0
                continue
            np.testing.assert_allclose(out["alpha"][r], al, rtol=1e-9)
            np.testing.assert_allclose(out["depth"][r] / out["alpha"][r], res.x, rtol=1e-6)


@pytest.mark.parametrize("which", ["pinhole", "fisheye", "lidar"])
def test_tiled_equals_brute_force(which):
    """Tile lists change nothing: tiled compositing == all particles in (key, index) order
    gated by rect membership, bit for bit in FP64."""
    if which == "pinhole":
        g, s = synth.scene_pinhole_small(2)
    elif which == "fisheye":
        g, s = synth.scene_fisheye(1, n=3000, width=160, height=112)
        g["mean"] *= np.float32(0.2)
    else:
        g, s = synth.scene_lidar(1, n=4000, n_beams=32, n_az=256, n_phi=4, max_per_tile=32)
        g["mean"] *= np.float32(0.1)
    proj, lists, out = oracle.render(g, s)
    assert lists["n_pairs"] > 100
    out_b = oracle.composite(g, s, lists, proj, mode=1)
    for k in out:
        assert np.array_equal(out[k], out_b[k]), k


def test_invariants_and_monotone_transmittance():
    g, s = synth.scene_pinhole_small(3)
    proj, lists, out = oracle.render(g, s)
    assert np.all((out["t_final"] >= 0) & (out["t_final"] <= 1))
    assert np.all((out["alpha"] >= 0) & (out["alpha"] <= 1))
    np.testing.assert_allclose(out["alpha"], 1 - out["t_final"], atol=1e-13)
    cmax = oracle.project(g, s)["feat"].max()
    assert np.all(out["feat"] <= cmax * out["alpha"] + 1e-12)
    # T over list prefixes is non-increasing (no early stop so prefixes are comparable)
    prev = np.ones(s["width"] * s["height"])
    r = lists["ranges"].copy()
    length = (r[1] - r[0]).max()
    for k in range(0, int(length) + 1, 4):
        lk = dict(lists)
        lk["ranges"] = np.stack([r[0], np.minimum(r[1], r[0] + k)])
        o = oracle.composite(g, s, lk, proj, t_min=0.0)
        assert np.all(o["t_final"] <= prev + 1e-15)
        prev = o["t_final"]


def test_permutation_invariance():
    g, s = synth.scene_pinhole_small(4)
    _, _, out = oracle.render(g, s)
    perm = np.random.default_rng(0).permutation(g["mean"].shape[1])
    _, _, out_p = oracle.render(synth.permute(g, perm), s)
    for k in out:
        assert np.array_equal(out[k], out_p[k]), k


def test_sort_order_and_ranges():
    g, s = synth.scene_pinhole_small(5)
    proj = oracle.project(g, s)
    lists = oracle.bin_pairs(s, proj["rect"], proj["count"], proj["key"])
    pairs = []
    TX = (s["width"] + 15) // 16
    for i in np.nonzero(proj["count"])[0]:
        x0, y0, x1, y1 = proj["rect"][:, i]
        for y in range(y0, y1 + 1):
            for x in range(x0, x1 + 1):
                pairs.append((y * TX + x, int(proj["key"][i]), int(i)))
    pairs.sort()
    assert [p[0] for p in pairs] == list(lists["pair_tile"])
    assert [p[2] for p in pairs] == list(lists["pair_gauss"])
    for t in range(lists["ranges"].shape[1]):
        a, b = lists["ranges"][:, t]
        assert all(p[0] == t for p in pairs[a:b])
        assert sum(p[0] == t for p in pairs) == b - a


def test_depth_key_is_float32_squared_distance():
    g, s = synth.scene_pinhole_small(6)
    s["origin"] = np.array([0.1, -0.2, 0.3], np.float32)
    proj = oracle.project(g, s)
    d = g["mean"] - s["origin"][:, None]
    key = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    assert np.array_equal(proj["key"], key.astype(np.float32).view(np.uint32))


def test_camera_rect_matches_brute_force_overlap():
    """Rect = the set of tiles whose pixel range meets [m - 3 sd, m + 3 sd]."""
    g, s = synth.scene_pinhole_small(7)
    proj = oracle.project(g, s)
    TX, TY = 8, 6
    for i in range(g["mean"].shape[1]):
        m, c = proj["mean2"][:, i], proj["cov2"][:, i]
        e = 3 * np.sqrt([c[0], c[2]])
        tiles = [(x, y) for y in range(TY) for x in range(TX)
                 if 16 * x <= m[0] + e[0] and 16 * (x + 1) > m[0] - e[0]
                 and 16 * y <= m[1] + e[1] and 16 * (y + 1) > m[1] - e[1]]
        x0, y0, x1, y1 = proj["rect"][:, i]
        got = [(x, y) for y in range(y0, y1 + 1) for x in range(x0, x1 + 1)] if proj["count"][i] else []
        assert sorted(got) == sorted(tiles)


# ------------------------------------------------------------------ LiDAR tiling and culling
@pytest.mark.parametrize("name", ["alg1_8beam.json", "alg1_multicross.json"])
def test_alg1_hand_worked(name):
    fx = json.load(open(os.path.join(GOLDEN, name)))
    be = np.deg2rad(np.array(fx["beam_elev_deg"])).astype(np.float32)
    bounds, bstart, nth = oracle.lidar_tiling(be, fx["n_az"], fx["n_phi"], fx["M"])
    np.testing.assert_allclose(np.rad2deg(bounds), fx["bounds_deg"], atol=1e-5)
    assert list(bstart) == fx["beam_start"]
    assert nth == fx["n_theta"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_alg1_invariants(seed):
    rng = np.random.default_rng(seed)
    be = synth.beams_uniform(rng, 128)
    A, NP, M = 2048, 16, 32
    bounds, bstart, nth = oracle.lidar_tiling(be, A, NP, M)
    assert bounds[0] == np.float64(be.min()) and abs(bounds[-1] - be.max()) < 1e-12
    assert np.all(np.diff(bounds) >= 0)
    counts = np.diff(bstart)
    assert counts.sum() == 128 and bstart[0] == 0
    # per-tile beam counts deviate from B/N_phi by at most the beams of one histogram bin
    w = (be.max() - be.min()) / 400
    bins = np.minimum(((be.astype(np.float64) - be.min()) / w).astype(int), 399)
    biggest_bin = np.bincount(bins).max()
    assert np.all(np.abs(counts - 128 / NP) <= biggest_bin + 1)
    assert nth == int(np.ceil(counts.max() * A / M))
    # every ray tile holds at most M (1 + 1/N_theta) rays
    per_az = [len([a for a in range(A) if a * nth // A == j]) for j in range(nth)]
    assert counts.max() * max(per_az) <= M * (1 + 1 / nth) + counts.max()


def test_sat_query_matches_mask_sum():
    rng = np.random.default_rng(8)
    be = synth.beams_uniform(rng, 24)
    mask, sat = oracle.ray_sat(be, 300, float(be.min()), float(be.max()), 160, 40)
    assert mask.sum() > 0
    for _ in range(500):
        x0, x1 = sorted(rng.integers(0, 160, 2))
        y0, y1 = sorted(rng.integers(0, 40, 2))
        n = sat[x1 + 1, y1 + 1] - sat[x0, y1 + 1] - sat[x1 + 1, y0] + sat[x0, y0]
        assert n == mask[x0:x1 + 1, y0:y1 + 1].sum()


def test_ray_culling_between_beams():
    """Alg. 2 / Alg. 3: a small particle that falls between two distant beams is culled;
    one on a beam is kept; culling never drops a particle some ray passes through."""
    be = np.deg2rad([-10.0, -9.9, 9.9, 10.0]).astype(np.float32)
    s = synth.lidar(be, 512, n_phi=2, max_per_tile=64, cull=True, cull_az=1600, cull_el_per_tile=8)
    mean = np.array([[50.0, 50.0 * np.cos(np.deg2rad(10.0))], [0.0, 0.0], [0.0, 50.0 * np.sin(np.deg2rad(10.0))]])
    g = synth.particles(np.random.default_rng(0), mean, 0.05, 0.05, 0, synth.FEAT_LIDAR)
    proj = oracle.project(g, s)
    assert proj["count"][0] == 0 and proj["n_culled_rays"] == 1
    assert proj["count"][1] > 0
    s_off = dict(s)
    s_off["cull"] = False
    assert oracle.project(g, s_off)["count"][0] > 0


def test_lidar_drop_probability_is_softmax():
    g, s = synth.scene_lidar(0, n=3000, n_beams=16, n_az=128, n_phi=4, max_per_tile=32)
    g["mean"] *= np.float32(0.05)
    proj, lists, out = oracle.render(g, s)
    z = out["feat"]
    ref = 1.0 / (1.0 + np.exp(-(z[2] - z[1])))
    np.testing.assert_allclose(out["drop"], ref, atol=1e-15)
    assert (out["alpha"] > 0).sum() > 50


# ------------------------------------------------------------------ gradients
def _small_diff_scene(seed, n=300, size=32, f=20.0):
    rng = np.random.default_rng(seed)
    mean = np.stack([rng.uniform(-3, 3, n), rng.uniform(-3, 3, n), rng.uniform(3, 9, n)])
    g = synth.particles(rng, mean, 0.05, 0.6, 3, synth.FEAT_CAMERA)
    return g, synth.pinhole(size, size, f, f, R_sw=synth.yaw_camera_pose(0.0) @ synth.yaw_camera_pose(0.0).T,
                            origin=[0.05, -0.02, 0.01])


def test_adjoint_matches_finite_differences_camera():
    g, s = _small_diff_scene(0)
    proj, lists, out = oracle.render(g, s)
    rng = np.random.default_rng(1)
    R = s["width"] * s["height"]
    up = dict(feat=rng.standard_normal((3, R)), depth=0.1 * rng.standard_normal(R),
              alpha=rng.standard_normal(R))
    gr = oracle.backward(g, s, lists, up)
    sel = np.nonzero(proj["count"])[0][:40]
    fd = oracle.fd_grad(g, s, lists, up, sel, h=1e-5)
    an = oracle.grads_as_rows(gr, sel)
    scale = np.abs(fd).max(axis=0, keepdims=True) + 1e-12
    assert np.abs(an).max() > 0
    np.testing.assert_allclose(an, fd, atol=1e-6 * scale.max(), rtol=1e-5)


def _thin_disc_scene(seed, n=500):
    """Discs 1e-3 to 1e-4 as thick as they are wide, 10-30 m in front of a 48x40 pinhole."""
    rng = np.random.default_rng(seed)
    mean = np.stack([rng.uniform(-4, 4, n), rng.uniform(-3, 3, n), rng.uniform(10, 30, n)])
    g = synth.particles(rng, mean, 0.3, 1.2, 0, synth.FEAT_CAMERA)
    w = rng.uniform(np.log(0.3), np.log(1.2), n)
    g["log_scale"] = np.stack([w, w + rng.uniform(-0.5, 0.5, n),
                               w + rng.uniform(np.log(1e-4), np.log(1e-3), n)]).astype(np.float32)
    return g, synth.pinhole(48, 40, 60.0, 60.0), rng


def test_adjoint_matches_finite_differences_thin_discs():
    """Thin particles: B's largest eigenvalue is 1e6-1e8 times its smallest, so the chain from
    dL/dB to rotation and scales must not pass through dL/dSigma = -B G B (whose entries reach
    (1/s_min^2)^2 |G|): that route is off by ~1% in the quaternion gradient here."""
    g, s, rng = _thin_disc_scene(11)
    R = s["width"] * s["height"]
    up = dict(feat=rng.standard_normal((3, R)), depth=0.1 * rng.standard_normal(R),
              alpha=rng.standard_normal(R))
    proj, lists, out = oracle.render(g, s)
    gr = oracle.backward(g, s, lists, up)
    sel = np.argsort(np.abs(gr["quat"]).sum(0))[-40:]
    fd = oracle.fd_grad(g, s, lists, up, sel, h=1e-5)
    an = oracle.grads_as_rows(gr, sel)
    geo = slice(0, 10)                               # mean, quat, log_scale
    scale = np.abs(fd[:, geo]).max()
    assert scale > 1.0
    np.testing.assert_allclose(an[:, geo], fd[:, geo], atol=1e-4 * scale, rtol=1e-4)


@pytest.mark.parametrize("theta", [0.0, 0.02])
def test_adjoint_matches_finite_differences_lidar(theta):
    """theta > 0: with the beam-divergence filter the mean also moves the smoothing term
    (r tan(theta/2))^2 (I - d d^T); finite differences see it through the full render."""
    g, s = synth.scene_lidar(2, n=2000, n_beams=16, n_az=128, n_phi=4, max_per_tile=32)
    g["mean"] *= np.float32(0.05)
    s["beam_divergence"] = theta
    proj, lists, out = oracle.render(g, s)
    rng = np.random.default_rng(2)
    R = out["alpha"].shape[0]
    up = dict(feat=rng.standard_normal((3, R)), depth=0.1 * rng.standard_normal(R),
              alpha=rng.standard_normal(R), drop=rng.standard_normal(R))
    gr = oracle.backward(g, s, lists, up)
    sel = np.nonzero(proj["count"])[0][:40]
    fd = oracle.fd_grad(g, s, lists, up, sel, h=1e-5)
    an = oracle.grads_as_rows(gr, sel)
    assert np.abs(an).max() > 0
    np.testing.assert_allclose(an, fd, atol=1e-6 * np.abs(fd).max(), rtol=1e-5)


# ------------------------------------------------------------------ time-dependent sensors
def _moving_pinhole(W=48, H=40, f=40.0, shift=(0.4, -0.1, 0.3), yaw=0.15):
    R0 = synth.yaw_camera_pose(0.3)
    R1 = synth.yaw_camera_pose(0.3 + yaw)
    o0 = np.array([0.5, -0.2, 0.1], np.float32)
    s = synth.pinhole(W, H, f, f, R_sw=R0, origin=o0)
    return synth.rolling_shutter(s, R1, o0 + np.asarray(shift, np.float32))


def test_moving_pose_matches_scipy_slerp():
    """The oracle's pose interpolation (quaternions from the matrices, shorter-arc slerp,
    linear origin) equals scipy's Slerp on the same float32 poses."""
    from scipy.spatial.transform import Slerp
    rng = np.random.default_rng(3)
    for _ in range(5):
        R0 = Rotation.random(random_state=rng).as_matrix().astype(np.float32)
        R1 = Rotation.random(random_state=rng).as_matrix().astype(np.float32)
        o0, o1 = rng.normal(size=3).astype(np.float32), rng.normal(size=3).astype(np.float32)
        s = synth.rolling_shutter(synth.pinhole(8, 8, 8.0, 8.0, R_sw=R0, origin=o0), R1, o1)
        sl = Slerp([0, 1], Rotation.from_matrix(np.stack([R0, R1]).astype(np.float64)))
        for t in (0.0, 0.13, 0.5, 0.77, 1.0):
            R, o = oracle.pose_at(s, t)
            # the float32 matrices are orthonormal only to ~1e-8; scipy projects them onto
            # rotations, the oracle normalises the extracted quaternion
            np.testing.assert_allclose(R, sl([t]).as_matrix()[0], atol=5e-8)
            np.testing.assert_allclose(o, (1 - t) * o0.astype(np.float64) + t * o1.astype(np.float64), atol=1e-14)


def test_rolling_shutter_ray_tables_round_trip():
    """A point on the ray of pixel (x, y), captured at t = (y + 0.5)/H from o(t), projects back
    to that pixel centre at the fixed point of the time-dependent projection (the generator
    builds the rays with scipy's Slerp, the oracle with its own interpolation)."""
    s = _moving_pinhole()
    s["rs_iters"] = 40                                  # converged fixed point
    d = s["ray_dir"].astype(np.float64)
    o = s["ray_org"].astype(np.float64)
    pts = (o + 6.0 * d).T
    uv, ok = oracle.project_points(s, pts)
    W = s["width"]
    idx = np.arange(d.shape[1])
    centre = np.stack([idx % W + 0.5, idx // W + 0.5], 1)
    assert ok.all()
    assert np.abs(uv - centre).max() < 2e-3             # float32 ray rounding


def test_spinning_lidar_ray_tables_round_trip():
    """Same for a spinning LiDAR in motion: column a fires at t = a / n_az; away from the
    sweep's seam a point on a ray projects back to its (azimuth, elevation)."""
    rng = np.random.default_rng(4)
    be = synth.beams_uniform(rng, 8, -15, 10)
    s = synth.lidar(be, 64, R_sw=synth.yaw_lidar_pose(0.7), origin=[1.0, 0.5, 0.2], n_phi=2, max_per_tile=16)
    s = synth.spinning(s, synth.yaw_lidar_pose(0.9), np.array([2.0, 0.8, 0.2], np.float32))
    s["rs_iters"] = 40
    d = s["ray_dir"].astype(np.float64)
    o = s["ray_org"].astype(np.float64)
    uv, ok = oracle.project_points(s, (o + 9.0 * d).T)
    a = np.tile(np.arange(64), 8)
    b = np.repeat(np.arange(8), 64)
    keep = (a > 1) & (a < 62)
    assert ok.all()
    np.testing.assert_allclose(uv[keep, 0], 2 * np.pi * a[keep] / 64, atol=2e-6)
    np.testing.assert_allclose(uv[keep, 1], np.sort(be).astype(np.float64)[b[keep]], atol=2e-6)


def test_moving_sensor_without_motion_equals_static():
    """A 'moving' camera whose two poses coincide renders what the static camera renders."""
    g, s = synth.scene_pinhole_small(3, n=600)
    m = synth.rolling_shutter(s, s["R_sw"], s["origin"])
    _, la, a = oracle.render(g, s)
    _, lb, b = oracle.render(g, m)
    assert la["n_pairs"] == lb["n_pairs"] and np.array_equal(la["pair_gauss"], lb["pair_gauss"])
    for k in ("feat", "depth", "alpha"):   # the moving table's rays differ by float32 rounding
        np.testing.assert_allclose(a[k], b[k], rtol=2e-6, atol=1e-6)


def test_per_ray_origin_closed_form():
    """One isotropic particle seen by a translating rolling-shutter camera: every ray uses its
    own origin, alpha_i = sigma exp(-|(mu - o_i) x d_i|^2 / (2 s^2)) (Eq. 1, 3D response)."""
    s = synth.pinhole(48, 48, 45.0, 45.0)
    s = synth.rolling_shutter(s, s["R_sw"], np.array([0.25, 0.0, 0.0], np.float32))
    mu = np.array([[0.1], [-0.05], [3.0]])
    g = synth.particles(np.random.default_rng(0), mu, 0.2, 0.2, 0, synth.FEAT_CAMERA,
                        dc=synth.camera_rgb_dc(np.array([[0.9], [0.4], [0.2]])))
    g["log_scale"][:] = np.float32(np.log(0.2))
    g["opacity_logit"][:] = np.float32(np.log(0.3 / 0.7))
    sigma = 1.0 / (1.0 + np.exp(-np.float64(g["opacity_logit"][0])))
    sc = np.exp(np.float64(g["log_scale"][0, 0]))
    _, lists, out = oracle.render(g, s)
    d = s["ray_dir"].astype(np.float64).T
    v = mu.ravel().astype(np.float32).astype(np.float64)[None] - s["ray_org"].astype(np.float64).T
    dd = np.sum(d * d, axis=1)
    tau = np.sum(v * d, axis=1) / dd
    D2 = np.sum(np.cross(v, d) ** 2, axis=1) / (sc**2 * dd)
    alpha = np.minimum(sigma * np.exp(-0.5 * D2), 0.99)
    alpha = np.where(alpha < 1 / 255, 0.0, alpha)
    hit = out["n_proc"] > 0
    assert (alpha > 0).sum() > 100 and np.all(alpha[~hit] == 0)
    np.testing.assert_allclose(out["alpha"], alpha, atol=1e-13)
    np.testing.assert_allclose(out["depth"], tau * alpha, atol=1e-12)


# ------------------------------------------------------------------ LiDAR beam divergence
def _divergence_scene(theta):
    rng = np.random.default_rng(8)
    be = synth.beams_uniform(rng, 32, -3, 4)
    s = synth.lidar(be, 2048, n_phi=2, max_per_tile=32)
    s["beam_divergence"] = theta
    mu = np.array([[6.0], [0.8], [0.1]])
    g = synth.particles(rng, mu, 0.05, 0.05, 0, synth.FEAT_LIDAR)
    g["feat"] = synth.lidar_feat(rng, 1)
    g["quat"][:, 0] = [1, 0, 0, 0]
    g["opacity_logit"][:] = np.float32(np.log(0.6 / 0.4))
    return g, s


def test_beam_divergence_response_is_numeric_maximum_of_the_smoothed_gaussian():
    """Eq. 6 reading: Sigma_hat = Sigma + (r tan(theta/2))^2 (I - d d^T) and alpha = sigma max_t
    exp(-q(t)/2) with no opacity factor; checked ray by ray against a bounded scalar maximisation
    of the smoothed density built here from that definition."""
    theta = 0.02
    g, s = _divergence_scene(theta)
    _, _, out = oracle.render(g, s)
    mu = g["mean"][:, 0].astype(np.float64)
    sc = np.exp(np.float64(g["log_scale"][0, 0]))
    r = np.linalg.norm(mu)
    d = mu / r
    w2 = (r * np.tan(theta / 2)) ** 2
    Sig = sc * sc * np.eye(3) + w2 * (np.eye(3) - np.outer(d, d))
    B = np.linalg.inv(Sig)
    sigma = 1 / (1 + np.exp(-np.float64(g["opacity_logit"][0])))
    dirs = s["ray_dir"].astype(np.float64).T
    hit = np.nonzero(out["alpha"] > 0)[0]
    assert len(hit) > 20
    for k in hit[:: max(1, len(hit) // 40)]:
        e = dirs[k]
        f = lambda t: (t * e - mu) @ B @ (t * e - mu)
        best = minimize_scalar(f, bounds=(0.1, 20.0), method="bounded", options={"xatol": 1e-12})
        a = min(sigma * np.exp(-0.5 * best.fun), 0.99)
        assert abs(out["alpha"][k] - a) < 1e-9 * max(1.0, a)
    # Coverage of the widened footprint (pins the sigma points built from the Cholesky factor):
    # every ray whose smoothed response clearly exceeds the cut-off must be composited.
    eb, mb = dirs @ B, B @ mu
    ebe = np.einsum("ij,ij->i", eb, dirs)
    qmin = mu @ mb - (eb @ mu) ** 2 / ebe
    front = (eb @ mu) / ebe > s["near"]          # the maximising point lies ahead of the sensor
    strong = np.nonzero(front & (sigma * np.exp(-0.5 * qmin) > 0.05))[0]
    assert len(strong) > 20 and np.all(out["alpha"][strong] > 0)


def test_beam_divergence_widens_without_scaling_opacity():
    """The filter widens the footprint (more rays hit) but keeps the peak: without an opacity
    factor the ray nearest the centre still sees alpha close to sigma (a determinant-ratio factor
    would scale it by about 0.41 here); theta = 0 is the plain response."""
    g, s0 = _divergence_scene(0.0)
    _, _, a0 = oracle.render(g, s0)
    g, s1 = _divergence_scene(0.02)
    _, _, a1 = oracle.render(g, s1)
    _, _, a_plain = oracle.render(g, {k: v for k, v in s0.items() if k != "beam_divergence"})
    np.testing.assert_array_equal(a0["alpha"], a_plain["alpha"])
    assert (a1["alpha"] > 0).sum() > 1.5 * (a0["alpha"] > 0).sum()
    sigma = 1 / (1 + np.exp(-np.float64(g["opacity_logit"][0])))
    assert a0["alpha"].max() <= a1["alpha"].max() <= sigma
    assert a1["alpha"].max() > 0.9 * sigma


# ------------------------------------------------------------------ rigid actor transforms
def _actor_case(seed=0, n_bg=300, n_actors=5, per_actor=40):
    from oracle import actors as oa
    rng = np.random.default_rng(seed)
    g, _ = synth.scene_pinhole_small(seed, n=n_bg)
    g, ids, poses = synth.actors(rng, g, n_actors, per_actor, [[-2, 2], [-1, 1], [3, 6]], up_axis=1)
    poses = poses.astype(np.float64)
    poses[:, :4] = rng.standard_normal((n_actors, 4))          # general (unnormalised) rotations
    ids[rng.choice(len(ids), 7, replace=False)] = n_actors + 3  # out-of-range ids: background
    return oa, g, ids, poses


def test_actor_transform_matches_scipy_rigid_motion():
    """mu_w = R_a mu + t and Sigma_w = R_a Sigma R_a^T, with R_a, R(q) and the composed rotation
    all from scipy (quaternion product not used on this side)."""
    from scipy.spatial.transform import Rotation
    oa, g, ids, poses = _actor_case()
    w = oa.actor_transform(g, ids, poses)
    n = len(ids)
    xyzw = lambda q: np.array([q[1], q[2], q[3], q[0]])
    for i in range(n):
        mu = g["mean"][:, i].astype(np.float64)
        q = g["quat"][:, i].astype(np.float64)
        S2 = np.diag(np.exp(2 * g["log_scale"][:, i].astype(np.float64)))
        Sig = Rotation.from_quat(xyzw(q)).as_matrix() @ S2 @ Rotation.from_quat(xyzw(q)).as_matrix().T
        Sig_w = Rotation.from_quat(xyzw(w["quat"][:, i])).as_matrix() @ S2 @ \
            Rotation.from_quat(xyzw(w["quat"][:, i])).as_matrix().T
        a = ids[i]
        if 0 <= a < len(poses):
            Ra = Rotation.from_quat(xyzw(poses[a, :4]))
            np.testing.assert_allclose(w["mean"][:, i], Ra.apply(mu) + poses[a, 4:], rtol=0, atol=1e-12)
            Rm = Ra.as_matrix()
            np.testing.assert_allclose(Sig_w, Rm @ Sig @ Rm.T, rtol=0, atol=1e-12 * np.abs(Sig).max())
            np.testing.assert_allclose(np.linalg.norm(w["quat"][:, i]), np.linalg.norm(q), rtol=1e-14)
        else:
            assert np.array_equal(w["mean"][:, i], mu) and np.array_equal(w["quat"][:, i], q)


def test_actor_transform_identity_and_composition():
    """The identity pose changes nothing; two successive poses equal their composition."""
    from scipy.spatial.transform import Rotation
    oa, g, ids, poses = _actor_case(1)
    ident = np.tile([1.0, 0, 0, 0, 0, 0, 0], (len(poses), 1))
    w = oa.actor_transform(g, ids, ident)
    np.testing.assert_allclose(w["mean"], g["mean"], atol=1e-15)
    np.testing.assert_allclose(w["quat"], g["quat"], atol=1e-15)
    rng = np.random.default_rng(5)
    p2 = np.concatenate([rng.standard_normal((len(poses), 4)), rng.standard_normal((len(poses), 3))], 1)
    two = oa.actor_transform(oa.actor_transform(g, ids, poses), ids, p2)
    xyzw = lambda q: np.array([q[1], q[2], q[3], q[0]])
    comp = np.zeros_like(poses)
    for a in range(len(poses)):
        R1, R2 = Rotation.from_quat(xyzw(poses[a, :4])), Rotation.from_quat(xyzw(p2[a, :4]))
        q = (R2 * R1).as_quat()
        comp[a, :4] = [q[3], q[0], q[1], q[2]]
        comp[a, 4:] = R2.apply(poses[a, 4:]) + p2[a, 4:]
    one = oa.actor_transform(g, ids, comp)
    np.testing.assert_allclose(two["mean"], one["mean"], atol=1e-12)
    # quaternions agree up to sign (q and -q are the same rotation)
    dots = np.abs(np.sum(two["quat"] * one["quat"], 0)) / np.sum(one["quat"] ** 2, 0)
    np.testing.assert_allclose(dots, 1.0, atol=1e-12)


def test_actor_transform_adjoint_matches_central_differences():
    oa, g, ids, poses = _actor_case(2, n_bg=20, n_actors=3, per_actor=6)
    rng = np.random.default_rng(3)
    n = len(ids)
    gm, gq = rng.standard_normal((3, n)), rng.standard_normal((4, n))
    dm, dq, dp = oa.actor_transform_backward(g, ids, poses, gm, gq)
    base = {k: np.asarray(v, np.float64) for k, v in g.items() if k in ("mean", "quat")}

    def f(mean, quat, P):
        w = oa.actor_transform(dict(g, mean=mean, quat=quat), ids, P)
        return np.sum(w["mean"] * gm) + np.sum(w["quat"] * gq)
    h = 1e-6
    for name, arr, ref in (("mean", base["mean"], dm), ("quat", base["quat"], dq), ("pose", poses, dp)):
        fd = np.zeros_like(arr)
        for idx in np.ndindex(arr.shape):
            ap, am = arr.copy(), arr.copy()
            ap[idx] += h
            am[idx] -= h
            args = lambda x: (x, base["quat"], poses) if name == "mean" else \
                ((base["mean"], x, poses) if name == "quat" else (base["mean"], base["quat"], x))
            fd[idx] = (f(*args(ap)) - f(*args(am))) / (2 * h)
        np.testing.assert_allclose(ref, fd, atol=1e-7 * np.abs(fd).max(), rtol=1e-6, err_msg=name)


def test_actor_render_invariant_under_common_rigid_motion():
    """Moving every particle with one actor pose and the sensor by the same motion leaves the
    image unchanged (SH degree 0: the colour has no direction to rotate)."""
    from oracle import actors as oa
    from scipy.spatial.transform import Rotation
    g, s = synth.scene_pinhole_small(4, n=800)
    ids = np.zeros(g["mean"].shape[1], np.int32)
    Ra = Rotation.from_rotvec([0.3, -0.5, 0.2])
    q = Ra.as_quat()
    pose = np.array([[q[3], q[0], q[1], q[2], 1.5, -0.5, 2.0]])
    gw = oa.actor_transform_f32(g, ids, pose)
    Rm = Ra.as_matrix()
    s_w = synth.pinhole(s["width"], s["height"], s["fx"], s["fy"],
                        R_sw=np.asarray(s["R_sw"], np.float64) @ Rm.T,
                        origin=Rm @ np.asarray(s["origin"], np.float64) + pose[0, 4:])
    _, _, a = oracle.render(g, s)
    _, _, b = oracle.render(gw, s_w)
    for k in ("feat", "depth", "alpha"):
        d = np.abs(np.asarray(a[k]) - np.asarray(b[k])) / max(1.0, np.abs(a[k]).max())
        assert np.mean(d) < 1e-6 and np.quantile(d, 0.995) < 1e-4, (k, d.max())
    assert (a["alpha"] > 0).mean() > 0.3
