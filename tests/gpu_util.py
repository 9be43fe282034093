"""Shared helpers of the GPU parity tests: run the HIP path through the C-ABI binding and
compare it with the oracle element by element."""
from __future__ import annotations

import numpy as np

import oracle

AMBIG = 1e-9          # decisions closer than this to their threshold are ambiguous
TOL = 1e-4            # max-abs bound on feat / depth / alpha / drop

REC_DTYPE = np.dtype([("b", "<f8", 6), ("bv", "<f8", 3), ("vbv", "<f8"), ("log_sigma", "<f8"), ("v", "<f8", 3),
                      ("feat", "<f4", 3), ("pad", "<f4")])


def rec_B(rec, i):
    """The symmetric 3x3 B of record i from its six unique entries."""
    b = rec["b"][i]
    return np.array([[b[0], b[1], b[2]], [b[1], b[3], b[4]], [b[2], b[4], b[5]]])


def to_np(t):
    return t.detach().cpu().numpy()


def gpu_render(g_np, s_np, moments=True, state=True):
    import torch
    import paper_2510_12901_amd as ut
    g = ut.GaussianSet.from_numpy(g_np)
    s = ut.Sensor(s_np)
    p, bins, out = ut.render(g, s, moments=moments, state=state)
    lists = ut.tile_lists(p, s, bins)
    torch.cuda.synchronize()
    P = lists.n_pairs
    res = dict(
        count=to_np(p.count).view(np.uint32)[:g.n], rect=to_np(p.rect)[:, :g.n], key=to_np(p.key).view(np.uint32)[:g.n],
        moments=to_np(p.moments)[:, :g.n] if moments else None, n_culled=to_np(p.n_culled),
        records=to_np(p.records)[: g.n * REC_DTYPE.itemsize].view(REC_DTYPE), gauss=to_np(lists.gauss).view(np.uint32)[:P],
        ranges=to_np(lists.ranges).view(np.uint32), n_pairs=P, n_bin_pairs=bins.n_pairs,
        feat=to_np(out.feat), depth=to_np(out.depth), alpha=to_np(out.alpha),
        drop=to_np(out.drop) if out.drop is not None else None,
        t_final=to_np(out.t_final) if out.t_final is not None else None,
        n_proc=to_np(out.n_proc).view(np.uint32) if out.n_proc is not None else None)
    return res, (g, s, p, bins, out)


def same_ranges(a, b):
    """[start, end) tile ranges describe the same lists: equal lengths, equal starts wherever
    a tile is non-empty (an empty range may sit at any offset)."""
    la, lb = a[1].astype(np.int64) - a[0], b[1].astype(np.int64) - b[0]
    return np.array_equal(la, lb) and np.array_equal(a[0][la > 0], b[0][lb > 0])


def ambiguous_tiles(op, gp, n_tiles, tiles_x, lidar):
    """Tiles touched (in either rect) by particles whose projection decisions are within
    AMBIG of a threshold."""
    bad = np.nonzero(op["margin"] < AMBIG)[0]
    tiles = set()
    for i in bad:
        for rect, cnt in ((op["rect"][:, i], op["count"][i]), (gp["rect"][:, i], gp["count"][i])):
            if cnt == 0:
                continue
            x0, y0, x1, y1 = rect
            for y in range(y0, y1 + 1):
                for x in range(x0, x1 + 1):
                    tiles.add(y * tiles_x + (x % tiles_x if lidar else x))
    return bad, tiles


def ray_tiles(osens):
    """Tile id of every ray (same mapping as the oracle)."""
    c = osens.c
    if osens.kind != 2:
        idx = np.arange(osens.n_rays)
        return (idx // c.width // c.tile) * osens.tiles_x + (idx % c.width) // c.tile
    b = np.repeat(np.arange(c.n_beams), c.n_az)
    a = np.tile(np.arange(c.n_az), c.n_beams)
    k = np.searchsorted(osens.beam_start[1:-1], b, side="right")
    return k * osens.tiles_x + (a * c.n_theta) // c.n_az


def compare_projection(gp, op, lidar):
    ok = op["margin"] >= AMBIG
    assert np.array_equal(gp["count"][ok], op["count"][ok])
    vis = ok & (op["count"] > 0)
    assert np.array_equal(gp["rect"][:, vis], op["rect"][:, vis])
    assert np.array_equal(gp["key"], op["key"])
    v = ok & (op["valid"] == 1)
    m = gp["moments"]
    ref = np.concatenate([op["mean2"], op["cov2"]])
    assert np.all(np.abs(m[:, v] - ref[:, v]) <= 1e-5 * (np.abs(ref[:, v]) + 1.0))
    vis = v & (gp["count"] > 0)            # records are written for particles that reach a tile
    assert np.abs(gp["records"]["feat"][vis].T - op["feat"][:, vis]).max(initial=0) <= 1e-6
    return int((~ok).sum())


def d2_representation_error(g_np):
    """Bound on the difference of two float64 evaluations of D^2 = u^T B u that start from
    different roundings of B.  An entry of B is rounded at its largest eigenvalue, 1/s_min^2,
    and a pair that reaches alpha_min has |u| <= 3.3 s_max (D^2 <= 2 ln(1/alpha_min) ~ 11), so
    the two D^2 differ by at most ~9 |u|^2 * 2 ulp(1/s_min^2) = 16 eps (3.3 s_max / s_min)^2
    (rounded up).  Negligible for ordinary particles, it is what separates two correct
    renders of particles 1e-4 as thick as they are wide."""
    sc = np.exp(np.asarray(g_np["log_scale"], np.float64))
    k = (3.3 * sc.max(axis=0) / sc.min(axis=0)) ** 2
    return float(16.0 * np.finfo(np.float64).eps * k.max())


def compare_outputs(go, oo, exclude_rays=None, tol=TOL, eps_d2=0.0):
    """eps_d2: per-pair D^2 difference allowed by the arithmetic (d2_representation_error);
    a composited pair moves ln T by alpha/(1-alpha) * eps_d2 / 2 <= 49.5 eps_d2."""
    keep = oo["margin"] >= AMBIG
    if exclude_rays is not None:
        keep &= ~exclude_rays
    errs = {}
    for k in ("feat", "depth", "alpha", "drop"):
        if oo.get(k) is None:
            continue
        d = np.abs(np.asarray(go[k], np.float64) - oo[k])
        d = d[..., keep]
        errs[k] = float(d.max(initial=0))
        assert errs[k] <= tol, (k, errs[k])
    assert np.array_equal(go["n_proc"][keep], oo["n_proc"][keep])
    t_ref = oo["t_final"][keep]
    t_tol = 1e-9 + (1e-9 + 49.5 * eps_d2 * oo["n_proc"][keep]) * t_ref
    assert np.all(np.abs(go["t_final"][keep] - t_ref) <= t_tol)
    return errs, int((~keep).sum())


def full_parity(g_np, s_np, eps_d2=0.0):
    """GPU pipeline vs oracle pipeline on a small scene; returns (errors, excluded rays).
    eps_d2 widens the t_final check for scenes of very thin particles (compare_outputs)."""
    gp, handles = gpu_render(g_np, s_np)
    os_ = oracle.OracleSensor(s_np)
    op, ol, oo = oracle.render(g_np, os_)
    n_amb = compare_projection(gp, op, os_.kind == 2)
    # the lists: oracle binning of the GPU's own rects / counts / keys must be identical
    ol_g = oracle.bin_pairs(os_, gp["rect"], gp["count"], gp["key"])
    assert gp["n_pairs"] == ol_g["n_pairs"]
    assert np.array_equal(gp["gauss"], ol_g["pair_gauss"])
    assert same_ranges(gp["ranges"], ol_g["ranges"])
    excl = None
    if n_amb:
        _, tiles = ambiguous_tiles(op, gp, os_.n_tiles, os_.tiles_x, os_.kind == 2)
        excl = np.isin(ray_tiles(os_), list(tiles))
    else:
        assert gp["n_pairs"] == ol["n_pairs"]
    errs, n_ex = compare_outputs(gp, oo, excl, eps_d2=eps_d2)
    return errs, n_ex, gp, oo, handles
