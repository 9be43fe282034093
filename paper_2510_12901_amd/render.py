"""Python binding of the C-ABI: device buffers are torch CUDA (HIP) tensors, every step of
the render runs in libutrast.so.  No CPU fallback exists; without the library or a GPU the
calls raise."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _abi as A
from ._abi import check, lib, ref

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4
UT_ABK = (1.0, 2.0, 0.0)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _require_cuda(t: torch.Tensor, dtype, name):
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")


# ---------------------------------------------------------------------------- particles
@dataclass
class GaussianSet:
    """Device-resident particles, structure-of-arrays float32 (see utrast.h)."""
    mean: torch.Tensor          # [3, N]
    quat: torch.Tensor          # [4, N]
    log_scale: torch.Tensor     # [3, N]
    opacity_logit: torch.Tensor  # [N]
    feat: torch.Tensor          # [K, 3, N]
    sh_degree: int
    feat_kind: int

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    @classmethod
    def from_numpy(cls, g: dict, device="cuda") -> "GaussianSet":
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=device)
        return cls(t(g["mean"]), t(g["quat"]), t(g["log_scale"]), t(g["opacity_logit"]), t(g["feat"]),
                   int(g["sh_degree"]), int(g["feat_kind"]))

    def with_params(self, mean, quat, log_scale, opacity_logit, feat) -> "GaussianSet":
        return GaussianSet(mean, quat, log_scale, opacity_logit, feat, self.sh_degree, self.feat_kind)

    def c(self) -> A.UtGaussians:
        for name in ("mean", "quat", "log_scale", "opacity_logit", "feat"):
            _require_cuda(getattr(self, name), torch.float32, name)
        return A.UtGaussians(self.mean.data_ptr(), self.quat.data_ptr(), self.log_scale.data_ptr(),
                             self.opacity_logit.data_ptr(), self.feat.data_ptr(), self.n,
                             self.sh_degree, self.feat_kind)


# ---------------------------------------------------------------------------- sensors
class Sensor:
    """A sensor definition with its device ray table and (LiDAR) tiling/culling tables,
    built once (ut_sensor_build) and reused across renders."""

    def __init__(self, desc: dict, device="cuda"):
        self.desc = desc
        c = A.UtSensor()
        c.kind = int(desc["kind"])
        c.R_sw[:] = [float(x) for x in np.asarray(desc["R_sw"], np.float32).ravel()]
        c.origin[:] = [float(x) for x in np.asarray(desc["origin"], np.float32)]
        c.near_ = float(desc.get("near", 0.1))
        self.ray_dir = torch.as_tensor(np.ascontiguousarray(desc["ray_dir"], np.float32), device=device)
        c.ray_dir = self.ray_dir.data_ptr()
        self.ray_org = None
        if desc.get("moving"):
            self.ray_org = torch.as_tensor(np.ascontiguousarray(desc["ray_org"], np.float32), device=device)
            c.moving = 1
            c.R_sw1[:] = [float(x) for x in np.asarray(desc["R_sw1"], np.float32).ravel()]
            c.origin1[:] = [float(x) for x in np.asarray(desc["origin1"], np.float32)]
            c.ray_org = self.ray_org.data_ptr()
            c.rs_iters = int(desc.get("rs_iters", 3))
        self._keep = []
        if c.kind == A.LIDAR:
            be = np.ascontiguousarray(desc["beam_elev"], np.float32)
            self._keep.append(be)
            c.beam_elev_host = be.ctypes.data
            c.n_beams, c.n_az = len(be), int(desc["n_az"])
            c.n_phi, c.max_per_tile = int(desc["n_phi"]), int(desc["max_per_tile"])
            c.cull = int(bool(desc.get("cull", True)))
            c.cull_az, c.cull_el = int(desc.get("cull_az", 1600)), int(desc.get("cull_el", 8 * c.n_phi))
            c.beam_divergence = float(desc.get("beam_divergence", 0.0))
        else:
            c.width, c.height = int(desc["width"]), int(desc["height"])
            c.fx, c.fy, c.cx, c.cy = (float(desc[k]) for k in ("fx", "fy", "cx", "cy"))
            c.k[:] = [float(x) for x in desc.get("k", [0, 0, 0, 0])]
            c.theta_max = float(desc.get("theta_max", 0.0))
        nb = C.c_size_t(0)
        check(lib().ut_sensor_table_bytes(ref(c), C.byref(nb)), "ut_sensor_table_bytes")
        self.tables = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=device)
        c.tables = self.tables.data_ptr()
        check(lib().ut_sensor_build(ref(c), _stream()), "ut_sensor_build")
        self.c = c
        self.kind = c.kind
        self.n_tiles = int(lib().ut_sensor_tiles(ref(c)))
        self.n_super = int(lib().ut_sensor_super_tiles(ref(c)))
        self.n_rays = int(lib().ut_sensor_rays(ref(c)))
        self.max_tile_rays = int(c.max_tile_rays)

    @property
    def is_lidar(self) -> bool:
        return self.kind == A.LIDAR

    def image_shape(self):
        if self.is_lidar:
            return (self.c.n_beams, self.c.n_az)
        return (self.c.height, self.c.width)


def lidar_tiling(beam_elev, n_az, n_phi, M):
    be = np.ascontiguousarray(beam_elev, np.float32)
    bounds = np.zeros(n_phi + 1, np.float64)
    bstart = np.zeros(n_phi + 1, np.int32)
    nth = C.c_int32(0)
    check(lib().ut_lidar_tiling(be.ctypes.data, len(be), n_az, n_phi, M, bounds.ctypes.data,
                                bstart.ctypes.data, C.byref(nth)), "ut_lidar_tiling")
    return bounds, bstart, int(nth.value)


# ---------------------------------------------------------------------------- stages
@dataclass
class Projection:
    records: torch.Tensor
    rect: torch.Tensor
    key: torch.Tensor
    count: torch.Tensor
    trect: torch.Tensor
    moments: torch.Tensor | None
    n_culled: torch.Tensor
    n: int
    _c: A.UtProjected = field(default=None, repr=False)

    def c(self) -> A.UtProjected:
        if self._c is None:
            self._c = A.UtProjected(self.records.data_ptr(), self.rect.data_ptr(), self.key.data_ptr(),
                                    self.count.data_ptr(), self.trect.data_ptr(),
                                    self.moments.data_ptr() if self.moments is not None else None,
                                    self.n_culled.data_ptr())
        return self._c


def alloc_projection(n: int, device="cuda", moments=False) -> Projection:
    nn = max(n, 1)
    return Projection(torch.empty(nn * A.RECORD_BYTES, dtype=torch.uint8, device=device),
                      torch.empty((4, nn), dtype=torch.int32, device=device),
                      torch.empty(nn, dtype=torch.int32, device=device),
                      torch.empty(nn, dtype=torch.int32, device=device),
                      torch.empty((nn, 2), dtype=torch.int32, device=device),
                      torch.empty((5, nn), dtype=torch.float32, device=device) if moments else None,
                      torch.empty(2, dtype=torch.int32, device=device), n)


def project(g: GaussianSet, sensor: Sensor, abk=UT_ABK, moments=False, out: Projection | None = None,
            stream=None) -> Projection:
    p = out if out is not None else alloc_projection(g.n, g.mean.device, moments)
    gc = g.c()
    abk_arr = (C.c_double * 3)(*abk)
    check(lib().ut_project(ref(gc), ref(sensor.c), C.cast(abk_arr, C.c_void_p), ref(p.c()), _stream(stream)),
          "ut_project")
    return p


@dataclass
class BinLists:
    """Super-tile bins: gauss ordered by (super-tile, depth key, index), ranges [2, n_super]."""
    gauss: torch.Tensor
    ranges: torch.Tensor
    n_pairs: int
    _c: A.UtBinLists = field(default=None, repr=False)

    def c(self) -> A.UtBinLists:
        if self._c is None:
            self._c = A.UtBinLists(self.gauss.data_ptr(), self.ranges.data_ptr(), int(self.gauss.numel()))
        return self._c


@dataclass
class TileLists:
    """Per-tile lists: gauss ordered by (tile, depth key, index), ranges [2, n_tiles]."""
    gauss: torch.Tensor
    ranges: torch.Tensor
    n_pairs: int
    total: torch.Tensor = None
    _c: A.UtTileLists = field(default=None, repr=False)

    def c(self) -> A.UtTileLists:
        if self._c is None:
            self._c = A.UtTileLists(self.gauss.data_ptr(), self.ranges.data_ptr(), int(self.gauss.numel()),
                                    self.total.data_ptr())
        return self._c


class Workspace:
    """Growable device workspace; growth keeps the leading bytes (the count stage's results)."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = torch.empty(256, dtype=torch.uint8, device=device)

    def ensure(self, nbytes: int, keep: int = 0) -> torch.Tensor:
        if self.buf.numel() < nbytes:
            new = torch.empty(int(nbytes * 1.25) + 256, dtype=torch.uint8, device=self.device)
            if keep:
                new[:keep].copy_(self.buf[:keep])
            self.buf = new
        return self.buf


_default_ws: dict = {}


def _ws(key) -> Workspace:
    key = str(key)
    if key not in _default_ws:
        _default_ws[key] = Workspace(key.split("/")[0])
    return _default_ws[key]


def bin_and_sort(p: Projection, sensor: Sensor, ws: Workspace | None = None, pair_ws: Workspace | None = None,
                 stream=None) -> BinLists:
    """Two-phase binning: count (pair total read back), then sort into exact-size bins."""
    dev = p.records.device
    ws = ws or _ws(dev)
    pair_ws = pair_ws or _ws(str(dev) + "/pairs")
    L = lib()
    buf = ws.ensure(int(L.ut_count_workspace_bytes(p.n)))
    total = torch.zeros(1, dtype=torch.int64).pin_memory()
    st = _stream(stream)
    check(L.ut_bin_count(ref(p.c()), p.n, ref(sensor.c), buf.data_ptr(), buf.numel(), total.data_ptr(), st),
          "ut_bin_count")
    (stream or torch.cuda.current_stream()).synchronize()
    P = int(total.item())
    pbuf = pair_ws.ensure(int(L.ut_pair_workspace_bytes(P)))
    bins = BinLists(torch.empty(max(P, 1), dtype=torch.int32, device=dev),
                    torch.empty((2, sensor.n_super), dtype=torch.int32, device=dev), P)
    check(L.ut_bin_sort(ref(p.c()), p.n, ref(sensor.c), buf.data_ptr(), buf.numel(), pbuf.data_ptr(), pbuf.numel(),
                        P, ref(bins.c()), st), "ut_bin_sort")
    return bins


def tile_lists(p: Projection, sensor: Sensor, bins: BinLists, stream=None) -> TileLists:
    """Materialise the per-tile (depth, index)-ordered lists from the bins."""
    dev = p.records.device
    L = lib()
    st = _stream(stream)
    tot_dev = torch.zeros(1, dtype=torch.int64, device=dev)
    lists = TileLists(torch.empty(1, dtype=torch.int32, device=dev),
                      torch.empty((2, sensor.n_tiles), dtype=torch.int32, device=dev), 0, tot_dev)
    host = torch.zeros(1, dtype=torch.int64).pin_memory()
    check(L.ut_tile_lists_count(ref(p.c()), ref(sensor.c), ref(bins.c()), ref(lists.c()), host.data_ptr(), st),
          "ut_tile_lists_count")
    (stream or torch.cuda.current_stream()).synchronize()
    P = int(host.item())
    lists = TileLists(torch.empty(max(P, 1), dtype=torch.int32, device=dev), lists.ranges, P, tot_dev)
    check(L.ut_tile_lists_fill(ref(p.c()), ref(sensor.c), ref(bins.c()), ref(lists.c()), st), "ut_tile_lists_fill")
    return lists


def render_params(alpha_min=ALPHA_MIN, alpha_max=ALPHA_MAX, t_min=T_MIN) -> A.UtRenderParams:
    return A.UtRenderParams(alpha_min, alpha_max, t_min)


@dataclass
class RenderOut:
    feat: torch.Tensor      # [3, R]
    depth: torch.Tensor     # [R]
    alpha: torch.Tensor     # [R]
    drop: torch.Tensor | None
    t_final: torch.Tensor | None
    n_proc: torch.Tensor | None
    n_visit: torch.Tensor | None = None     # work counters (optional)
    n_pass: torch.Tensor | None = None
    tile_end: torch.Tensor | None = None    # adjoint state: per tile, the bin index past its last entry
    _c: A.UtRenderOut = field(default=None, repr=False)

    def c(self) -> A.UtRenderOut:
        if self._c is None:
            self._c = A.UtRenderOut(self.feat.data_ptr(), self.depth.data_ptr(), self.alpha.data_ptr(),
                                    _ptr(self.drop), _ptr(self.t_final), _ptr(self.n_proc),
                                    _ptr(self.n_visit), _ptr(self.n_pass), _ptr(self.tile_end))
        return self._c


def alloc_out(sensor: Sensor, device="cuda", state=True, counters=False) -> RenderOut:
    R = sensor.n_rays
    return RenderOut(torch.empty((3, R), dtype=torch.float32, device=device),
                     torch.empty(R, dtype=torch.float32, device=device),
                     torch.empty(R, dtype=torch.float32, device=device),
                     torch.empty(R, dtype=torch.float32, device=device) if sensor.is_lidar else None,
                     torch.empty(R, dtype=torch.float64, device=device) if state else None,
                     torch.empty(R, dtype=torch.int32, device=device) if state else None,
                     torch.empty(R, dtype=torch.int32, device=device) if counters else None,
                     torch.empty(R, dtype=torch.int32, device=device) if counters else None,
                     torch.empty(max(sensor.n_tiles, 1), dtype=torch.int32, device=device) if state else None)


def composite(p: Projection, bins: BinLists, sensor: Sensor, params=None, out: RenderOut | None = None,
              state=True, stream=None) -> RenderOut:
    o = out if out is not None else alloc_out(sensor, p.records.device, state)
    prm = params or render_params()
    fn = lib().ut_composite_lidar if sensor.is_lidar else lib().ut_composite_camera
    check(fn(ref(p.c()), ref(bins.c()), ref(sensor.c), ref(prm), ref(o.c()), _stream(stream)), "ut_composite")
    return o


def render(g: GaussianSet, sensor: Sensor, abk=UT_ABK, params=None, state=True, moments=False, stream=None):
    """project -> bin_and_sort -> composite; returns (projection, bins, outputs)."""
    p = project(g, sensor, abk, moments=moments, stream=stream)
    bins = bin_and_sort(p, sensor, stream=stream)
    out = composite(p, bins, sensor, params, state=state, stream=stream)
    return p, bins, out


def backward(g: GaussianSet, p: Projection, bins: BinLists, sensor: Sensor, fwd: RenderOut,
             up_feat=None, up_depth=None, up_alpha=None, up_drop=None, params=None, stream=None) -> dict:
    """Adjoint: gradients of sum(upstream * outputs) with respect to the particle parameters.
    ``bins`` are the forward's super-tile bins; ``fwd`` its outputs with the adjoint state."""
    dev = g.mean.device
    if not isinstance(bins, BinLists):
        raise TypeError("backward takes the forward's BinLists")
    if fwd.t_final is None or fwd.n_proc is None or fwd.tile_end is None:
        raise ValueError("the forward must be rendered with state=True")
    prm = params or render_params()
    acc = torch.empty(int(lib().ut_backward_workspace_bytes(g.n)), dtype=torch.uint8, device=dev)
    grads = dict(mean=torch.empty_like(g.mean), quat=torch.empty_like(g.quat),
                 log_scale=torch.empty_like(g.log_scale), opacity_logit=torch.empty_like(g.opacity_logit),
                 feat=torch.empty_like(g.feat))
    gg = A.UtGaussianGrads(*(grads[k].data_ptr() for k in ("mean", "quat", "log_scale", "opacity_logit", "feat")))
    keep = [t.contiguous().float() if t is not None else None for t in (up_feat, up_depth, up_alpha, up_drop)]
    up = A.UtUpstream(*(_ptr(t) for t in keep))
    gc = g.c()
    check(lib().ut_composite_backward(ref(gc), ref(p.c()), ref(bins.c()), ref(sensor.c), ref(prm), ref(fwd.c()),
                                      ref(up), acc.data_ptr(), acc.numel(), ref(gg), _stream(stream)),
          "ut_composite_backward")
    return grads


def composite_batch(items, params=None, n_workgroups=0, ws: torch.Tensor | None = None, stream=None):
    """One launch compositing several (projection, lists, sensor, out) requests: one workgroup
    per (request, tile) item (n_workgroups = 0, the default), or that many persistent
    workgroups looping over the items."""
    n = len(items)
    prm = params or render_params()
    arr = (A.UtBatchItem * n)()
    keep = []
    for i, (p, bins, sensor, out) in enumerate(items):
        pc, lc, oc = p.c(), bins.c(), out.c()
        keep += [pc, lc, oc]
        arr[i] = A.UtBatchItem(ref(pc), ref(lc), ref(sensor.c), ref(oc))
    need = int(lib().ut_batch_workspace_bytes(n))
    dev = items[0][0].records.device
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    check(lib().ut_composite_batch(C.cast(arr, C.c_void_p), n, ref(prm), ws.data_ptr(), ws.numel(), n_workgroups, _stream(stream)),
          "ut_composite_batch")
    return ws


def composite_batch_noalloc(items, params=None, n_workgroups=None, stream=None):
    """composite_batch on the library's fixed per-GPU queue (ut_composite_batch_noalloc): no
    workspace, no device allocation.  Calls that overlap on one GPU race on that queue."""
    n = len(items)
    prm = params or render_params()
    arr = (A.UtBatchItem * n)()
    keep = []
    for i, (p, bins, sensor, out) in enumerate(items):
        pc, lc, oc = p.c(), bins.c(), out.c()
        keep += [pc, lc, oc]
        arr[i] = A.UtBatchItem(ref(pc), ref(lc), ref(sensor.c), ref(oc))
    check(lib().ut_composite_batch_noalloc(C.cast(arr, C.c_void_p), n, ref(prm),
                                           256 * 4 if n_workgroups is None else n_workgroups, _stream(stream)),
          "ut_composite_batch_noalloc")


class SensorPipeline:
    """Preallocated per-sensor render path: projection, two-phase binning and compositing
    with buffers reused across calls (no device allocation once the list capacity fits)."""

    def __init__(self, g: GaussianSet, sensor: Sensor, params=None, state=False, abk=UT_ABK):
        self.g, self.sensor, self.abk = g, sensor, abk
        dev = g.mean.device
        self.params = params or render_params()
        self.p = alloc_projection(g.n, dev)
        self.ws = Workspace(dev)
        self.pair_ws = Workspace(dev)
        self.out = alloc_out(sensor, dev, state=state)
        self.total = torch.zeros(1, dtype=torch.int64).pin_memory()
        self.bins: BinLists | None = None
        self.n_pairs = 0
        self.capacity = 0                 # pair capacity of the device-count path
        self.overflow = torch.zeros(1, dtype=torch.int32, device=dev)

    def _ensure_bins(self, P: int):
        dev = self.g.mean.device
        if self.bins is None or self.bins.gauss.numel() < P:
            self.bins = BinLists(torch.empty(max(int(P * 1.1), 1), dtype=torch.int32, device=dev),
                                 torch.empty((2, self.sensor.n_super), dtype=torch.int32, device=dev), P)
        self.bins.n_pairs = P

    def project(self, stream=None):
        """Stage a1 (+ a2): ut_project into the pipeline's projection buffers."""
        gc = self.g.c()
        abk_arr = (C.c_double * 3)(*self.abk)
        check(lib().ut_project(ref(gc), ref(self.sensor.c), C.cast(abk_arr, C.c_void_p), ref(self.p.c()),
                               _stream(stream)), "ut_project")

    def count(self, stream=None):
        """First half of binning: depth sort of the visible particles and the pair total."""
        L = lib()
        buf = self.ws.ensure(int(L.ut_count_workspace_bytes(self.g.n)))
        check(L.ut_bin_count(ref(self.p.c()), self.g.n, ref(self.sensor.c), buf.data_ptr(), buf.numel(),
                             self.total.data_ptr(), _stream(stream)), "ut_bin_count")

    def project_and_count(self, stream=None):
        self.project(stream)
        self.count(stream)

    def sort_and_composite(self, stream=None, composite_events=None):
        """Call after the count has completed on the host (stream synchronised)."""
        L = lib()
        st = _stream(stream)
        P = int(self.total.item())
        buf = self.ws.buf
        pbuf = self.pair_ws.ensure(int(L.ut_pair_workspace_bytes(P)))
        self._ensure_bins(P)
        self.n_pairs = P
        check(L.ut_bin_sort(ref(self.p.c()), self.g.n, ref(self.sensor.c), buf.data_ptr(), buf.numel(),
                            pbuf.data_ptr(), pbuf.numel(), P, ref(self.bins.c()), st), "ut_bin_sort")
        if composite_events is not None:
            composite_events[0].record(stream)
        fn = L.ut_composite_lidar if self.sensor.is_lidar else L.ut_composite_camera
        check(fn(ref(self.p.c()), ref(self.bins.c()), ref(self.sensor.c), ref(self.params), ref(self.out.c()), st),
              "ut_composite")
        if composite_events is not None:
            composite_events[1].record(stream)

    def set_capacity(self, max_pairs: int):
        """Size the bins and the pair workspace for the device-count path (no host round trip
        between counting and sorting); a frame whose pair total exceeds max_pairs raises the
        overflow flag and renders nothing."""
        max_pairs = int(max_pairs)
        self.pair_ws.ensure(int(lib().ut_pair_workspace_bytes(max_pairs)))
        self._ensure_bins(max_pairs)
        self.capacity = max_pairs

    def sort_and_composite_device(self, stream=None, composite_events=None):
        """Sort and composite right after project_and_count on the same stream, the pair total
        staying on the device (ut_bin_sort_device).  Check ``overflowed()`` once the stream has
        completed."""
        self.sort_device(stream)
        if composite_events is not None:
            composite_events[0].record(stream)
        self.composite_only(stream)
        if composite_events is not None:
            composite_events[1].record(stream)

    def sort_device(self, stream=None):
        """Second half of binning with the pair total kept on the GPU (ut_bin_sort_device)."""
        if self.capacity <= 0:
            raise ValueError("set_capacity first")
        buf = self.ws.buf
        pbuf = self.pair_ws.buf
        check(lib().ut_bin_sort_device(ref(self.p.c()), self.g.n, ref(self.sensor.c), buf.data_ptr(), buf.numel(),
                                       pbuf.data_ptr(), pbuf.numel(), self.capacity, ref(self.bins.c()),
                                       self.overflow.data_ptr(), _stream(stream)), "ut_bin_sort_device")

    def run_device(self, stream=None, composite_events=None):
        """One render with no host synchronisation (device-count path)."""
        s = stream or torch.cuda.current_stream()
        self.project_and_count(s)
        self.sort_and_composite_device(s, composite_events)
        return self.out

    def overflowed(self) -> bool:
        return bool(self.overflow.item())

    def clear_overflow(self):
        self.overflow.zero_()

    def composite_only(self, stream=None, out: RenderOut | None = None):
        L = lib()
        fn = L.ut_composite_lidar if self.sensor.is_lidar else L.ut_composite_camera
        o = out or self.out
        check(fn(ref(self.p.c()), ref(self.bins.c()), ref(self.sensor.c), ref(self.params), ref(o.c()),
                 _stream(stream)), "ut_composite")
        return o

    def run(self, stream=None, composite_events=None):
        s = stream or torch.cuda.current_stream()
        self.project_and_count(s)
        s.synchronize()
        self.sort_and_composite(s, composite_events)
        return self.out


class FrameGraph:
    """One frame of several sensor renders captured in a HIP graph (device-count path: no host
    round trip inside the frame).  Each pipeline runs on its own stream forked from the
    capture stream; replay() re-runs projection, binning, sort and compositing of every
    sensor into the pipelines' own output buffers.  Every pipeline must have its capacity set
    (SensorPipeline.set_capacity) and have run once eagerly (buffers sized); check the
    pipelines' overflowed() after a replay has completed."""

    def __init__(self, pipes, stream=None):
        if any(p.capacity <= 0 for p in pipes):
            raise ValueError("set_capacity on every pipeline before capturing")
        self.pipes = list(pipes)
        self.main = stream or torch.cuda.Stream()
        self.side = [torch.cuda.Stream() for _ in self.pipes]
        self.graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(self.graph, stream=self.main):
            fork = torch.cuda.Event()
            fork.record(self.main)
            joins = []
            for p, st in zip(self.pipes, self.side):
                st.wait_event(fork)
                p.project_and_count(st)
                p.sort_and_composite_device(st)
                e = torch.cuda.Event()
                e.record(st)
                joins.append(e)
            for e in joins:
                self.main.wait_event(e)
        torch.cuda.synchronize()

    def replay(self):
        self.graph.replay()

    def overflowed(self) -> bool:
        return any(p.overflowed() for p in self.pipes)


# ---------------------------------------------------------------------------- spatial order
def spatial_order(g: GaussianSet, stream=None) -> torch.Tensor:
    """int32 [N] permutation: the particle indices along the Z-order curve of their means
    (ut_spatial_order).  Reordering a resident scene once makes the projection's reads of the
    particles one view sees share cache lines."""
    dev = g.mean.device
    perm = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
    ws = torch.empty(int(lib().ut_spatial_order_workspace_bytes(g.n)), dtype=torch.uint8, device=dev)
    gc = g.c()
    check(lib().ut_spatial_order(ref(gc), _ptr(perm), _ptr(ws), ws.numel(), _stream(stream)), "ut_spatial_order")
    return perm[: g.n]


def gather(g: GaussianSet, perm: torch.Tensor, stream=None) -> GaussianSet:
    """The set reordered by perm (row j = source particle perm[j]), ut_gather_gaussians."""
    _require_cuda(perm, torch.int32, "perm")
    out = GaussianSet(torch.empty_like(g.mean), torch.empty_like(g.quat), torch.empty_like(g.log_scale),
                      torch.empty_like(g.opacity_logit), torch.empty_like(g.feat), g.sh_degree, g.feat_kind)
    gc = g.c()
    check(lib().ut_gather_gaussians(ref(gc), _ptr(perm), _ptr(out.mean), _ptr(out.quat), _ptr(out.log_scale),
                                    _ptr(out.opacity_logit), _ptr(out.feat), _stream(stream)), "ut_gather_gaussians")
    return out


# ---------------------------------------------------------------------------- scene graph
def actor_poses(poses) -> torch.Tensor:
    """Pose table [n_actors, 7] (qw, qx, qy, qz, tx, ty, tz) -> the device layout of
    ut_actor_pose, float32 [n_actors, 8] (last column unused)."""
    p = torch.as_tensor(poses, dtype=torch.float32)
    if p.dim() != 2 or p.shape[1] not in (7, 8):
        raise ValueError("poses must be [n_actors, 7]")
    if p.shape[1] == 7:
        p = torch.cat([p, torch.zeros_like(p[:, :1])], 1)
    return p.contiguous()


def actor_transform(g: GaussianSet, actor: torch.Tensor, poses: torch.Tensor, out: GaussianSet | None = None,
                    stream=None) -> GaussianSet:
    """World-frame copy of an object-frame particle set (ut_actor_transform): new mean and
    quaternion tensors (or those of ``out``, rewritten), the other arrays shared.  actor:
    int32 [N] on the device (-1 = background); poses: [n_actors, 7] or [n_actors, 8] float32."""
    _require_cuda(actor, torch.int32, "actor")
    poses = poses if poses.shape[-1] == 8 and poses.is_cuda else actor_poses(poses).to(g.mean.device)
    _require_cuda(poses, torch.float32, "poses")
    if out is not None:
        _require_cuda(out.mean, torch.float32, "out.mean")
        _require_cuda(out.quat, torch.float32, "out.quat")
        if out.mean.shape != g.mean.shape or out.quat.shape != g.quat.shape:
            raise ValueError("out must have the shape of g")
        mean_w, quat_w = out.mean, out.quat
    else:
        mean_w, quat_w = torch.empty_like(g.mean), torch.empty_like(g.quat)
    gc = g.c()
    check(lib().ut_actor_transform(ref(gc), _ptr(actor), _ptr(poses), int(poses.shape[0]), _ptr(mean_w),
                                   _ptr(quat_w), _stream(stream)), "ut_actor_transform")
    return out if out is not None else g.with_params(mean_w, quat_w, g.log_scale, g.opacity_logit, g.feat)


def actor_transform_backward(g: GaussianSet, actor: torch.Tensor, poses: torch.Tensor, d_mean_world: torch.Tensor,
                             d_quat_world: torch.Tensor, pose_grad: bool = True, stream=None):
    """Adjoint of actor_transform: (d_mean, d_quat) with respect to the object-frame set and
    the pose gradient float64 [n_actors, 7] (None when pose_grad is False)."""
    _require_cuda(actor, torch.int32, "actor")
    poses = poses if poses.shape[-1] == 8 and poses.is_cuda else actor_poses(poses).to(g.mean.device)
    dmw, dqw = d_mean_world.contiguous().float(), d_quat_world.contiguous().float()
    d_mean, d_quat = torch.empty_like(g.mean), torch.empty_like(g.quat)
    n_act = int(poses.shape[0])
    d_pose = torch.empty((n_act, 7), dtype=torch.float64, device=g.mean.device) if pose_grad else None
    gc = g.c()
    check(lib().ut_actor_transform_backward(ref(gc), _ptr(actor), _ptr(poses), n_act, _ptr(dmw), _ptr(dqw),
                                            _ptr(d_mean), _ptr(d_quat), _ptr(d_pose), _stream(stream)),
          "ut_actor_transform_backward")
    return d_mean, d_quat, d_pose

