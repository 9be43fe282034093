"""Pins of the oracle's LiDAR tile rect and ray-based culling (CPU).

The oracle turns a particle's UT moments into an azimuth-elevation tile rect (elevation
bands searched in the Alg. 1 boundaries, azimuth tiles by floor with a wrap modulo N_theta,
every tile once the extent spans a full turn) and, with culling on, into a range query on
the summed-area table of the ray mask (Sec. 3.3 "Tiling" and "Ray-based Culling";
Appendix A Alg. 1; Appendix B Alg. 2 and 3).  These tests state the same sets without
any of that index arithmetic:

* the rect is the set of tiles (band k, azimuth tile j) whose cell
  [T_k, T_{k+1}) x [2 pi j / N_theta, 2 pi (j + 1) / N_theta) meets the 3-sigma box
  [m_el - e_el, m_el + e_el] x ([m_az - e_az, m_az + e_az] modulo 2 pi) (the top band is
  closed above);
* a particle survives culling iff some culling cell that holds a ray meets the same box,
  where the cell of ray (b, a) is found from the beam's elevation and the ray's azimuth
  2 pi a / n_az, and cells are compared with the box as intervals.

Particles are drawn to reach the awkward cases: extents across azimuth 0, extents of a full
turn or more, and extents that end within 1e-9..1e-6 rad of an azimuth tile edge, an
elevation band edge or a culling-cell edge on either side.  Decisions closer than 1e-12 rad
to an azimuth or culling-cell edge are left out (the oracle finds those edges by a floor of
a product, the test by comparing with 2 pi j / N, and float64 rounding could go either way)
and counted; extents that end exactly on a band edge are kept, since both sides compare the
same float64 values there.
"""
import math

import numpy as np

import oracle
import synth

TWO_PI = 2.0 * math.pi
TIE = 1e-12


def _particles(mean, log_scale, quat=None, feat_rng=0):
    rng = np.random.default_rng(feat_rng)
    n = mean.shape[1]
    g = synth.particles(rng, np.asarray(mean, np.float64), 0.1, 0.1, 0, synth.FEAT_LIDAR)
    g["log_scale"] = np.ascontiguousarray(log_scale, np.float32)
    if quat is not None:
        g["quat"] = np.ascontiguousarray(quat, np.float32)
    g["feat"] = synth.lidar_feat(rng, n)
    return g


def _cyl(rho, phi, z):
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z])


def _box(proj, i):
    m_az, m_el = proj["mean2"][:, i]
    e_az = 3.0 * math.sqrt(proj["cov2"][0, i])
    e_el = 3.0 * math.sqrt(proj["cov2"][2, i])
    return m_az, e_az, m_el - e_el, m_el + e_el


def _az_meets(lo_cell, hi_cell, m, e):
    """Closed interval [m - e, m + e] taken modulo 2 pi meets the half-open [lo_cell, hi_cell)."""
    if 2.0 * e >= TWO_PI:
        return True
    return any(m - e < hi_cell + TWO_PI * w and m + e >= lo_cell + TWO_PI * w for w in range(-2, 3))


def _az_edge_distance(m, e, edges):
    d = math.inf
    for v in (m - e, m + e):
        for w in range(-2, 3):
            d = min(d, float(np.min(np.abs(edges + TWO_PI * w - v))))
    return d


def _brute_rect(m, e, lo, hi, T, n_theta):
    NP = len(T) - 1
    if hi < T[0] or lo > T[NP]:
        return set()
    tiles = set()
    for k in range(NP):
        top = lo <= T[k + 1] if k == NP - 1 else lo < T[k + 1]
        if not (top and hi >= T[k]):
            continue
        for j in range(n_theta):
            if _az_meets(TWO_PI * j / n_theta, TWO_PI * (j + 1) / n_theta, m, e):
                tiles.add((j, k))
    return tiles


def _oracle_rect(proj, i, n_theta):
    x0, y0, x1, y1 = (int(v) for v in proj["rect"][:, i])
    if proj["count"][i] == 0 and (x1 < x0 or y1 < y0):
        return set(), 0
    cells = [(x % n_theta, y) for y in range(y0, y1 + 1) for x in range(x0, x1 + 1)]
    return set(cells), len(cells)


def _rect_scene():
    """Sensor with 8 elevation bands; particles in five groups (see the module docstring)."""
    rng = np.random.default_rng(11)
    be = synth.beams_uniform(rng, 32, -30.0, 20.0)
    sensor = synth.lidar(be, 512, n_phi=8, max_per_tile=64, cull=False)
    so = oracle.OracleSensor(sensor)
    NT = so.c.n_theta
    groups, means, scales, quats = {}, [], [], []

    def add(name, mean, ls, q=None):
        n0 = sum(m.shape[1] for m in means)
        means.append(mean)
        scales.append(ls)
        quats.append(synth.unit_quaternions(rng, mean.shape[1]) if q is None else q)
        groups[name] = np.arange(n0, n0 + mean.shape[1])

    n = 500
    add("general", _cyl(rng.uniform(1, 80, n), rng.uniform(0, TWO_PI, n), rng.uniform(-10, 10, n)),
        rng.uniform(np.log(0.02), np.log(2.0), (3, n)))
    n = 120
    add("straddle", _cyl(rng.uniform(2, 20, n), rng.uniform(-0.05, 0.05, n), rng.uniform(-3, 3, n)),
        rng.uniform(np.log(0.05), np.log(0.5), (3, n)))
    n = 80
    ls = np.stack([rng.uniform(np.log(0.3), np.log(1.0), n), rng.uniform(np.log(0.02), np.log(0.1), n),
                   rng.uniform(np.log(0.02), np.log(0.1), n)])
    add("near_field", _cyl(rng.uniform(0.2, 0.6, n), rng.uniform(0, TWO_PI, n), rng.uniform(-0.15, 0.15, n)),
        ls, np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n)))
    # clouds whose extent ends next to an azimuth tile edge; isotropic particles, so the UT
    # azimuth mean is the particle's own azimuth and the extent does not depend on it
    rho, z, s = 10.0, 1.0, 0.1
    probe = oracle.project(_particles(_cyl(np.array([rho]), np.array([1.0]), np.array([z])),
                                      np.full((3, 1), np.log(s))), so)
    e_az = 3.0 * math.sqrt(probe["cov2"][0, 0])
    delta = np.concatenate([-np.logspace(-9, -6, 40), np.logspace(-9, -6, 40)])
    for j in (0, 1, NT // 2, NT - 1):
        edge = TWO_PI * j / NT
        for side in (-1.0, 1.0):          # -1: left end of the extent at the edge
            phi = edge - side * e_az + delta
            add(f"az_edge_{j}_{int(side)}", _cyl(np.full(phi.size, rho), phi, np.full(phi.size, z)),
                np.full((3, phi.size), np.log(s)))
    # clouds for the elevation band edges: same range and scale, heights stepped around h0
    # so that the low (or high) end of the extent sweeps across a value that a band edge
    # is then moved to
    h0 = [-2.0, 1.5]
    for c, h in enumerate(h0):
        hz = h + rho * np.concatenate([[0.0], rng.uniform(-1.5e-6, 1.5e-6, 299)])
        add(f"el_cloud_{c}", _cyl(np.full(hz.size, rho), np.full(hz.size, 0.7 + c), hz),
            np.full((3, hz.size), np.log(s)))
    mean = np.concatenate(means, 1)
    g = _particles(mean, np.concatenate(scales, 1), np.concatenate(quats, 1))
    # move two interior band edges onto the clouds' low / high extent ends
    first = oracle.project(g, so)
    ends = []
    for c in range(len(h0)):
        i = groups[f"el_cloud_{c}"][0]               # the cloud's unshifted particle
        _, _, lo, hi = _box(first, i)
        ends += [lo, hi]
    T = so.bounds
    inner = np.sort(np.concatenate([np.array(ends), np.linspace(T[0], T[-1], 8)[1:-1]]))
    assert inner[0] > T[0] and inner[-1] < T[-1] and inner.size >= 7
    keep = np.sort(np.concatenate([np.array(ends), inner[np.isin(inner, ends, invert=True)][:7 - len(ends)]]))
    T[1:-1] = keep                                   # the oracle reads the bounds in place
    assert np.all(np.diff(T) > 0)
    return g, so, groups


def test_lidar_rect_matches_brute_force_cell_overlap():
    g, so, groups = _rect_scene()
    proj = oracle.project(g, so)
    NT, T = so.c.n_theta, so.bounds
    az_edges = TWO_PI * np.arange(NT + 1) / NT
    checked, ties = 0, 0
    near = {(k, side): 0 for k in ("az_lo", "az_hi", "el_lo", "el_hi") for side in (-1, 1)}
    full_turn, wrapped, exact = 0, 0, 0
    for i in range(g["mean"].shape[1]):
        if not proj["valid"][i]:
            continue
        m, e, lo, hi = _box(proj, i)
        # the band edges are compared exactly as the oracle compares them (the same float64
        # values), so only azimuth decisions can be ties
        if _az_edge_distance(m, e, az_edges) < TIE:
            ties += 1
            continue
        want = _brute_rect(m, e, lo, hi, T, NT)
        got, n_cells = _oracle_rect(proj, i, NT)
        assert got == want, (i, m, e, lo, hi, sorted(got)[:8], sorted(want)[:8])
        assert n_cells == len(want) and int(proj["count"][i]) == len(want), i
        checked += 1
        full_turn += 2 * e >= TWO_PI and len(want) > 0
        wrapped += int(proj["rect"][2, i]) >= NT and len(want) > 0
        for name, v, edges in (("az_lo", m - e, az_edges), ("az_hi", m + e, az_edges),
                               ("el_lo", lo, T), ("el_hi", hi, T)):
            off = [v - x - TWO_PI * w for x in edges for w in ((-1, 0, 1) if edges is az_edges else (0,))]
            o = min(off, key=abs)
            if abs(o) < 1e-7:
                near[(name, 1 if o > 0 else -1)] += 1
            exact += name.startswith("el") and o == 0.0
    assert checked > 1000 and ties <= 4, (checked, ties)
    assert full_turn >= 3 and wrapped >= 20, (full_turn, wrapped)
    assert min(near.values()) >= 2, near          # each edge kind, from either side
    assert exact >= 4, exact                     # extents ending exactly on a band edge


def _brute_kept(m, e, lo, hi, occupied, T0, span, cull_az, cull_el):
    """Some occupied culling cell meets the box (cells and box compared as intervals)."""
    for ca, ce in occupied:
        el_lo = T0 + ce * span / cull_el
        el_hi = T0 + (ce + 1) * span / cull_el
        el_ok = (lo <= el_hi if ce == cull_el - 1 else lo < el_hi) and hi >= el_lo
        if el_ok and _az_meets(TWO_PI * ca / cull_az, TWO_PI * (ca + 1) / cull_az, m, e):
            return True
    return False


def test_lidar_culling_matches_cells_holding_rays():
    """Sparse beams and 256 azimuth steps leave most of the 1600 x 64 culling cells empty."""
    rng = np.random.default_rng(12)
    be = synth.beams_uniform(rng, 8, -20.0, 10.0)
    sensor = synth.lidar(be, 256, n_phi=8, max_per_tile=64, cull=True, cull_az=1600, cull_el_per_tile=8)
    so = oracle.OracleSensor(sensor)
    CA, CE = so.c.cull_az, so.c.cull_el
    T0, TN = so.bounds[0], so.bounds[-1]
    span = TN - T0
    # the cells that hold a ray, from each ray's own azimuth and its beam's elevation
    occupied = set()
    for b, eb in enumerate(so.beam_elev.astype(np.float64)):
        ce = min(max(int(math.floor((eb - T0) * CE / span)), 0), CE - 1)
        while ce + 1 < CE and eb >= T0 + (ce + 1) * span / CE:
            ce += 1
        while ce > 0 and eb < T0 + ce * span / CE:
            ce -= 1
        for a in range(256):
            occupied.add(((a * CA) // 256, ce))
    assert 0 < len(occupied) < CA * CE // 10
    # small particles scattered between the rays, plus clouds whose azimuth extent ends
    # next to the edge of an occupied cell whose neighbour is empty
    n = 1500
    el = rng.uniform(np.deg2rad(-21.0), np.deg2rad(11.0), n)
    rho = rng.uniform(5.0, 50.0, n)
    means = [np.stack([rho * np.cos(el) * np.cos(p), rho * np.cos(el) * np.sin(p), rho * np.sin(el)])
             for p in [rng.uniform(0, TWO_PI, n)]]
    scales = [rng.uniform(np.log(0.003), np.log(0.08), (3, n))]
    quats = [synth.unit_quaternions(rng, n)]
    rho_c, s_c, b_c = 20.0, 0.01, 3
    el_c = float(be[b_c])
    probe = oracle.project(_particles(np.array([[rho_c * math.cos(el_c)], [0.0], [rho_c * math.sin(el_c)]]),
                                      np.full((3, 1), np.log(s_c))), so)
    e_az = 3.0 * math.sqrt(probe["cov2"][0, 0])
    assert 2 * e_az < TWO_PI / CA, "cloud extents must fit inside one culling cell"
    delta = np.concatenate([-np.logspace(-9, -6, 30), np.logspace(-9, -6, 30)])
    for a in (0, 5, 128, 255):
        ca = (a * CA) // 256
        for side, edge in ((+1.0, TWO_PI * ca / CA), (-1.0, TWO_PI * (ca + 1) / CA)):
            # side +1: the right end of the extent at the cell's left edge
            phi = edge - side * e_az + delta
            means.append(np.stack([rho_c * math.cos(el_c) * np.cos(phi), rho_c * math.cos(el_c) * np.sin(phi),
                                   np.full(phi.size, rho_c * math.sin(el_c))]))
            scales.append(np.full((3, phi.size), np.log(s_c)))
            quats.append(np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, phi.size)))
    g = _particles(np.concatenate(means, 1), np.concatenate(scales, 1), np.concatenate(quats, 1))
    proj = oracle.project(g, so)
    cell_az = TWO_PI * np.arange(CA + 1) / CA
    cell_el = T0 + np.arange(CE + 1) * span / CE
    kept = culled = ties = near_kept = near_culled = 0
    for i in range(g["mean"].shape[1]):
        if not proj["valid"][i]:
            continue
        m, e, lo, hi = _box(proj, i)
        if hi < T0 or lo > TN:
            assert proj["count"][i] == 0
            continue
        d = min(_az_edge_distance(m, e, cell_az), float(np.min(np.abs(cell_el - lo))),
                float(np.min(np.abs(cell_el - hi))))
        if d < TIE:
            ties += 1
            continue
        want = _brute_kept(m, e, lo, hi, occupied, T0, span, CA, CE)
        assert (proj["count"][i] > 0) == want, (i, m, e, lo, hi, want)
        kept += want
        culled += not want
        if d < 1e-7:
            near_kept += want
            near_culled += not want
    assert ties <= 4 and kept > 200 and culled > 200, (ties, kept, culled)
    assert near_kept >= 8 and near_culled >= 8, (near_kept, near_culled)
    in_band = [i for i in range(g["mean"].shape[1]) if proj["valid"][i]
               and not (_box(proj, i)[3] < T0 or _box(proj, i)[2] > TN)]
    assert proj["n_culled_rays"] == sum(int(proj["count"][i] == 0) for i in in_band)
