"""ctypes shim of the FP64 CPU oracle (``utoracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``; never by the product package.  It takes the same
seeded float32 inputs as the GPU path (``synth``), converts them to float64 and calls the
oracle, which follows the paper step by step (see the comments in ``utoracle.cpp``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# UTORACLE_LIB: load a separately built copy instead (the sanitizer test's instrumented build)
LIB_PATH = os.environ.get("UTORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "utoracle.cpp")
CXXFLAGS = ["-O2", "-std=c++17", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
            "-fPIC", "-shared"]

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4
R_BINS = 400          # Alg. 1 histogram resolution
RS_ITERS = 3          # fixed-point iterations of the time-dependent projection (reading)


def build(force: bool = False) -> str:
    if os.environ.get("UTORACLE_LIB"):
        return LIB_PATH
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["g++", *CXXFLAGS, SRC_PATH, "-o", tmp])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Gaussians(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("quat", C.c_void_p), ("log_scale", C.c_void_p),
                ("opacity_logit", C.c_void_p), ("feat", C.c_void_p),
                ("n", C.c_int), ("sh_degree", C.c_int), ("feat_kind", C.c_int)]


class Sensor(C.Structure):
    _fields_ = [("kind", C.c_int), ("R_sw", C.c_float * 9), ("origin", C.c_float * 3),
                ("width", C.c_int), ("height", C.c_int), ("tile", C.c_int),
                ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("k", C.c_double * 4), ("theta_max", C.c_double), ("near_", C.c_double),
                ("n_beams", C.c_int), ("n_az", C.c_int), ("n_phi", C.c_int), ("n_theta", C.c_int),
                ("elev_bounds", C.c_void_p), ("beam_start", C.c_void_p),
                ("cull", C.c_int), ("cull_az", C.c_int), ("cull_el", C.c_int),
                ("sat", C.c_void_p), ("ray_dir", C.c_void_p),
                ("moving", C.c_int), ("R_sw1", C.c_float * 9), ("origin1", C.c_float * 3),
                ("ray_org", C.c_void_p), ("rs_iters", C.c_int), ("beam_divergence", C.c_double)]


class Params(C.Structure):
    _fields_ = [("ut_alpha", C.c_double), ("ut_beta", C.c_double), ("ut_kappa", C.c_double),
                ("alpha_min", C.c_double), ("alpha_max", C.c_double), ("t_min", C.c_double)]


class Projected(C.Structure):
    _fields_ = [("valid", C.c_void_p), ("mean2", C.c_void_p), ("cov2", C.c_void_p),
                ("rect", C.c_void_p), ("count", C.c_void_p), ("key", C.c_void_p),
                ("feat", C.c_void_p), ("margin", C.c_void_p),
                ("n_culled_invalid", C.c_int), ("n_culled_rays", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_lidar_tiling.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P, P, P]
        L.orc_ray_sat.argtypes = [P, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, P, P]
        L.orc_project.argtypes = [P, P, P, P]
        L.orc_count_pairs.argtypes = [P, C.c_int]
        L.orc_count_pairs.restype = C.c_uint64
        L.orc_bin.argtypes = [P, C.c_int, P, P, P, P, P, P]
        L.orc_composite.argtypes = [P, P, P, P, P, C.c_int, P, P, P, P, P, P, P, P, P, P]
        L.orc_composite_rays.argtypes = [P, P, P, P, P, P, C.c_int, P, P, P, P, P, P, P]
        L.orc_backward.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_fd_grad.argtypes = [P, P, P, P, P, P, P, P, P, P, C.c_int, C.c_double, P]
        L.orc_sh_eval.argtypes = [C.c_int, P, C.c_int, P]
        L.orc_pose_at.argtypes = [P, C.c_double, P, P]
        L.orc_project_points.argtypes = [P, P, C.c_int, P, P]
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class OracleGaussians:
    """float64 copies of a synth particle dict, kept alive with the ctypes view."""

    def __init__(self, g: dict):
        self.mean = _f64(g["mean"])
        self.quat = _f64(g["quat"])
        self.log_scale = _f64(g["log_scale"])
        self.opacity_logit = _f64(g["opacity_logit"])
        self.feat = _f64(g["feat"])
        self.n = self.mean.shape[1]
        self.sh_degree = int(g["sh_degree"])
        self.feat_kind = int(g["feat_kind"])
        self.c = Gaussians(_p(self.mean).value, _p(self.quat).value, _p(self.log_scale).value,
                           _p(self.opacity_logit).value, _p(self.feat).value,
                           self.n, self.sh_degree, self.feat_kind)


def lidar_tiling(beam_elev, n_az, n_phi, M, r_bins=R_BINS):
    be = np.ascontiguousarray(beam_elev, dtype=np.float32)
    bounds = np.zeros(n_phi + 1, np.float64)
    bstart = np.zeros(n_phi + 1, np.int32)
    nth = np.zeros(1, np.int32)
    rc = lib().orc_lidar_tiling(_p(be), len(be), n_az, n_phi, M, r_bins, _p(bounds), _p(bstart), _p(nth))
    if rc != 0:
        raise ValueError("invalid tiling arguments")
    return bounds, bstart, int(nth[0])


def ray_sat(beam_elev, n_az, emin, emax, cull_az, cull_el):
    be = np.ascontiguousarray(beam_elev, dtype=np.float32)
    mask = np.zeros((cull_az, cull_el), np.int32)
    sat = np.zeros((cull_az + 1, cull_el + 1), np.int32)
    lib().orc_ray_sat(_p(be), len(be), n_az, emin, emax, cull_az, cull_el, _p(mask), _p(sat))
    return mask, sat


class OracleSensor:
    """Oracle view of a synth sensor dict; LiDAR tiling and culling tables are computed
    here by the oracle's own Alg. 1 and summed-area table."""

    def __init__(self, s: dict):
        self.d = s
        self.ray_dir = np.ascontiguousarray(s["ray_dir"], dtype=np.float32)
        c = Sensor()
        c.kind = int(s["kind"])
        c.R_sw[:] = [float(x) for x in np.asarray(s["R_sw"], np.float32).ravel()]
        c.origin[:] = [float(x) for x in np.asarray(s["origin"], np.float32)]
        c.near_ = float(s.get("near", 0.1))
        c.ray_dir = _p(self.ray_dir).value
        if s.get("moving"):
            self.ray_org = np.ascontiguousarray(s["ray_org"], dtype=np.float32)
            c.moving = 1
            c.R_sw1[:] = [float(x) for x in np.asarray(s["R_sw1"], np.float32).ravel()]
            c.origin1[:] = [float(x) for x in np.asarray(s["origin1"], np.float32)]
            c.ray_org = _p(self.ray_org).value
            c.rs_iters = int(s.get("rs_iters", RS_ITERS))
        self.kind = c.kind
        if c.kind == 2:
            self.beam_elev = np.ascontiguousarray(s["beam_elev"], dtype=np.float32)
            n_phi, M = int(s["n_phi"]), int(s["max_per_tile"])
            self.bounds, self.beam_start, n_theta = lidar_tiling(self.beam_elev, s["n_az"], n_phi, M)
            c.n_beams, c.n_az, c.n_phi, c.n_theta = len(self.beam_elev), int(s["n_az"]), n_phi, n_theta
            c.elev_bounds = _p(self.bounds).value
            c.beam_start = _p(self.beam_start).value
            c.cull = int(bool(s.get("cull", True)))
            c.cull_az, c.cull_el = int(s["cull_az"]), int(s["cull_el"])
            self.mask, self.sat = ray_sat(self.beam_elev, c.n_az, self.bounds[0], self.bounds[-1],
                                          c.cull_az, c.cull_el)
            c.beam_divergence = float(s.get("beam_divergence", 0.0))
            c.sat = _p(self.sat).value
            self.n_tiles = n_phi * n_theta
            self.n_rays = c.n_beams * c.n_az
            self.tiles_x, self.tiles_y = n_theta, n_phi
        else:
            c.width, c.height, c.tile = int(s["width"]), int(s["height"]), int(s.get("tile", 16))
            c.fx, c.fy, c.cx, c.cy = float(s["fx"]), float(s["fy"]), float(s["cx"]), float(s["cy"])
            c.k[:] = [float(x) for x in s.get("k", [0, 0, 0, 0])]
            c.theta_max = float(s.get("theta_max", 0.0))
            self.tiles_x = (c.width + c.tile - 1) // c.tile
            self.tiles_y = (c.height + c.tile - 1) // c.tile
            self.n_tiles = self.tiles_x * self.tiles_y
            self.n_rays = c.width * c.height
        self.c = c


def make_params(abk=(1.0, 2.0, 0.0), alpha_min=ALPHA_MIN, alpha_max=ALPHA_MAX, t_min=T_MIN):
    return Params(float(abk[0]), float(abk[1]), float(abk[2]), alpha_min, alpha_max, t_min)


def _as_g(g):
    return g if isinstance(g, OracleGaussians) else OracleGaussians(g)


def _as_s(s):
    return s if isinstance(s, OracleSensor) else OracleSensor(s)


def project(g, s, abk=(1.0, 2.0, 0.0)) -> dict:
    g, s = _as_g(g), _as_s(s)
    n = g.n
    out = dict(valid=np.zeros(n, np.int32), mean2=np.zeros((2, n)), cov2=np.zeros((3, n)),
               rect=np.zeros((4, n), np.int32), count=np.zeros(n, np.uint32),
               key=np.zeros(n, np.uint32), feat=np.zeros((3, n)), margin=np.zeros(n))
    pr = Projected(*[_p(out[k]).value for k in ("valid", "mean2", "cov2", "rect", "count", "key", "feat", "margin")], 0, 0)
    prm = make_params(abk)
    lib().orc_project(C.byref(g.c), C.byref(s.c), C.byref(prm), C.byref(pr))
    out["n_culled_invalid"] = pr.n_culled_invalid
    out["n_culled_rays"] = pr.n_culled_rays
    return out


def bin_pairs(s, rect, count, key):
    s = _as_s(s)
    rect = np.ascontiguousarray(rect, np.int32)
    count = np.ascontiguousarray(count, np.uint32)
    key = np.ascontiguousarray(key, np.uint32)
    n = count.shape[0]
    P = int(lib().orc_count_pairs(_p(count), n))
    pt = np.zeros(max(P, 1), np.uint32)
    pg = np.zeros(max(P, 1), np.uint32)
    ranges = np.zeros((2, s.n_tiles), np.uint32)
    lib().orc_bin(C.byref(s.c), n, _p(rect), _p(count), _p(key), _p(pt), _p(pg), _p(ranges))
    return dict(pair_tile=pt[:P], pair_gauss=pg[:P], ranges=ranges, n_pairs=P)


def composite(g, s, lists, proj, mode=0, abk=(1.0, 2.0, 0.0), alpha_min=ALPHA_MIN,
              alpha_max=ALPHA_MAX, t_min=T_MIN) -> dict:
    g, s = _as_g(g), _as_s(s)
    R = s.n_rays
    out = dict(feat=np.zeros((3, R)), depth=np.zeros(R), alpha=np.zeros(R),
               t_final=np.zeros(R), n_proc=np.zeros(R, np.uint32), margin=np.zeros(R))
    drop = np.zeros(R) if s.kind == 2 else None
    pg = np.ascontiguousarray(lists["pair_gauss"], np.uint32)
    if pg.size == 0:
        pg = np.zeros(1, np.uint32)
    ranges = np.ascontiguousarray(lists["ranges"], np.uint32)
    rect = np.ascontiguousarray(proj["rect"], np.int32)
    count = np.ascontiguousarray(proj["count"], np.uint32)
    key = np.ascontiguousarray(proj["key"], np.uint32)
    prm = make_params(abk, alpha_min, alpha_max, t_min)
    lib().orc_composite(C.byref(g.c), C.byref(s.c), C.byref(prm), _p(pg), _p(ranges), mode,
                        _p(rect), _p(count), _p(key), _p(out["feat"]), _p(out["depth"]),
                        _p(out["alpha"]), _p(out["t_final"]), _p(out["n_proc"]),
                        _p(drop) if drop is not None else None, _p(out["margin"]))
    if drop is not None:
        out["drop"] = drop
    return out


def composite_rays(g, s, lists, ray_ids, abk=(1.0, 2.0, 0.0)) -> dict:
    """Composite only the given rays (for sampled checks of full-size renders)."""
    g, s = _as_g(g), _as_s(s)
    ids = np.ascontiguousarray(ray_ids, np.int64)
    m = len(ids)
    out = dict(feat=np.zeros((3, m)), depth=np.zeros(m), alpha=np.zeros(m), t_final=np.zeros(m),
               n_proc=np.zeros(m, np.uint32), margin=np.zeros(m))
    drop = np.zeros(m) if s.kind == 2 else None
    pg = np.ascontiguousarray(lists["pair_gauss"], np.uint32)
    if pg.size == 0:
        pg = np.zeros(1, np.uint32)
    ranges = np.ascontiguousarray(lists["ranges"], np.uint32)
    prm = make_params(abk)
    lib().orc_composite_rays(C.byref(g.c), C.byref(s.c), C.byref(prm), _p(pg), _p(ranges), _p(ids), m,
                             _p(out["feat"]), _p(out["depth"]), _p(out["alpha"]), _p(out["t_final"]),
                             _p(out["n_proc"]), _p(drop) if drop is not None else None, _p(out["margin"]))
    if drop is not None:
        out["drop"] = drop
    return out


def render(g, s, abk=(1.0, 2.0, 0.0), mode=0):
    """Full oracle pipeline: project -> bin -> composite."""
    g, s = _as_g(g), _as_s(s)
    proj = project(g, s, abk)
    lists = bin_pairs(s, proj["rect"], proj["count"], proj["key"])
    out = composite(g, s, lists, proj, mode=mode, abk=abk)
    return proj, lists, out


def _upstream(s, up):
    R = s.n_rays
    gf = _f64(up.get("feat", np.zeros((3, R))))
    gd = _f64(up.get("depth", np.zeros(R)))
    ga = _f64(up.get("alpha", np.zeros(R)))
    gdrop = _f64(up["drop"]) if "drop" in up else None
    return gf, gd, ga, gdrop


def backward(g, s, lists, upstream: dict, abk=(1.0, 2.0, 0.0)) -> dict:
    """Analytic FP64 gradient of sum(upstream * outputs) (frozen discrete structure)."""
    g, s = _as_g(g), _as_s(s)
    n, K = g.n, (g.sh_degree + 1) ** 2
    gf, gd, ga, gdrop = _upstream(s, upstream)
    out = dict(mean=np.zeros((3, n)), quat=np.zeros((4, n)), log_scale=np.zeros((3, n)),
               opacity_logit=np.zeros(n), feat=np.zeros((K, 3, n)))
    pg = np.ascontiguousarray(lists["pair_gauss"], np.uint32)
    if pg.size == 0:
        pg = np.zeros(1, np.uint32)
    ranges = np.ascontiguousarray(lists["ranges"], np.uint32)
    prm = make_params(abk)
    lib().orc_backward(C.byref(g.c), C.byref(s.c), C.byref(prm), _p(pg), _p(ranges), _p(gf), _p(gd),
                       _p(ga), _p(gdrop) if gdrop is not None else None, _p(out["mean"]),
                       _p(out["quat"]), _p(out["log_scale"]), _p(out["opacity_logit"]), _p(out["feat"]))
    return out


def fd_grad(g, s, lists, upstream: dict, sel, h=1e-4, abk=(1.0, 2.0, 0.0)) -> np.ndarray:
    """Central differences [len(sel), 11 + 3K]: mean(3), quat(4), log_scale(3), logit, feat(3K)."""
    g, s = _as_g(g), _as_s(s)
    K = (g.sh_degree + 1) ** 2
    gf, gd, ga, gdrop = _upstream(s, upstream)
    sel = np.ascontiguousarray(sel, np.int32)
    out = np.zeros((len(sel), 11 + 3 * K))
    pg = np.ascontiguousarray(lists["pair_gauss"], np.uint32)
    if pg.size == 0:
        pg = np.zeros(1, np.uint32)
    ranges = np.ascontiguousarray(lists["ranges"], np.uint32)
    prm = make_params(abk)
    lib().orc_fd_grad(C.byref(g.c), C.byref(s.c), C.byref(prm), _p(pg), _p(ranges), _p(gf), _p(gd),
                      _p(ga), _p(gdrop) if gdrop is not None else None, _p(sel), len(sel), h, _p(out))
    return out


def grads_as_rows(gr: dict, sel) -> np.ndarray:
    """Analytic gradients of the particles in ``sel`` laid out like ``fd_grad`` rows."""
    sel = np.asarray(sel)
    K = gr["feat"].shape[0]
    return np.concatenate([gr["mean"][:, sel].T, gr["quat"][:, sel].T, gr["log_scale"][:, sel].T,
                           gr["opacity_logit"][sel][:, None],
                           gr["feat"][:, :, sel].reshape(3 * K, -1).T], axis=1)


def sh_eval(deg, dirs):
    dirs = _f64(dirs).reshape(-1, 3)
    K = (deg + 1) ** 2
    Y = np.zeros((dirs.shape[0], K))
    lib().orc_sh_eval(deg, _p(dirs), dirs.shape[0], _p(Y))
    return Y


def project_points(s, pts):
    s = _as_s(s)
    pts = _f64(pts).reshape(-1, 3)
    uv = np.zeros((pts.shape[0], 2))
    ok = np.zeros(pts.shape[0], np.int32)
    lib().orc_project_points(C.byref(s.c), _p(pts), pts.shape[0], _p(uv), _p(ok))
    return uv, ok.astype(bool)


def pose_at(s, t: float):
    """(R_sw, origin) of a (moving) sensor at frame time t, as the oracle interpolates it."""
    s = _as_s(s)
    R = np.zeros(9)
    o = np.zeros(3)
    lib().orc_pose_at(C.byref(s.c), float(t), _p(R), _p(o))
    return R.reshape(3, 3), o


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(t: int) -> None:
    """OpenMP threads of the following oracle calls."""
    lib().orc_set_num_threads(int(t))
