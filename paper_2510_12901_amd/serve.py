"""Continuous-batching render server for closed-loop multi-sensor simulation.

The particle scene stays resident on the GPU.  Every request renders one sensor.  The host
loop moves each request through:

  waiting    arrived, no slot free yet
  counting   projection + pair count enqueued on the slot's own stream
  counted    pair total P known; waits until the device pool can hold its pair workspace and
             tile lists (admission by the memory its tile lists need)
  sorting    binning / radix sort enqueued on the slot stream
  batched    composited together with every other sorted request in one persistent launch
             (ut_composite_batch) on one of two compositing streams
  done       latency recorded; pool memory and slot released

Requests that arrive while others are on the GPU are admitted as slots and pool memory free
up, and their projection / sorting overlaps the compositing of earlier requests.  The
compositing arithmetic per ray is the single-request kernel's, so served outputs are
bit-identical to plain renders.
"""
from __future__ import annotations

import contextlib
import gc
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _abi as A
from ._abi import check, lib, ref
from .render import (BinLists, GaussianSet, RenderOut, Sensor, SensorPipeline, _stream, alloc_projection,
                     render_params)

ALIGN = 256


@contextlib.contextmanager
def _collector_paused():
    """Keep Python's cyclic garbage collector out of a serving loop.  A full (oldest
    generation) collection walks every object the process holds -- with torch and the scene
    loaded that is a pause of tens of milliseconds, long enough to stall every request in
    flight.  The loops create no reference cycles (their objects are freed by reference
    counting), so the collector is paused for the run and its previous state restored."""
    was = gc.isenabled()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()


class DevicePool:
    """First-fit allocator over one preallocated device buffer (host-side bookkeeping)."""

    def __init__(self, nbytes: int, device="cuda"):
        self.nbytes = int(nbytes)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.free = [(0, self.nbytes)]          # sorted (offset, size)
        self.in_use = 0
        self.peak = 0

    def alloc(self, n: int):
        n = (int(n) + ALIGN - 1) // ALIGN * ALIGN
        for i, (o, s) in enumerate(self.free):
            if s >= n:
                if s == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + n, s - n)
                self.in_use += n
                self.peak = max(self.peak, self.in_use)
                return (o, n)
        return None

    def release(self, blk):
        o, n = blk
        self.in_use -= n
        self.free.append((o, n))
        self.free.sort()
        merged = []
        for fo, fs in self.free:
            if merged and merged[-1][0] + merged[-1][1] == fo:
                merged[-1] = (merged[-1][0], merged[-1][1] + fs)
            else:
                merged.append((fo, fs))
        self.free = merged

    def view(self, blk, offset, nbytes):
        return self.buf[blk[0] + offset: blk[0] + offset + nbytes]


@dataclass
class Request:
    rid: int
    frame: int
    sensor: int
    arrival: float
    t_done: float = -1.0
    t_start: float = -1.0      # slot taken, projection enqueued
    t_counted: float = -1.0    # pair total seen on the host
    t_sort: float = -1.0       # pool memory granted, sort enqueued
    t_batch: float = -1.0      # compositing launch enqueued
    n_pairs: int = 0
    slot: "Slot" = None
    mem: tuple = None
    bins: BinLists = None
    out: RenderOut = None


class Slot:
    """Per-request-in-flight device state: a stream, projection buffers, count workspace,
    output buffers sized for the largest sensor, and its events."""

    def __init__(self, n: int, max_rays: int, device):
        self.stream = torch.cuda.Stream(device=device)
        self.p = alloc_projection(n, device)
        self.ws = torch.empty(int(lib().ut_count_workspace_bytes(n)), dtype=torch.uint8, device=device)
        self.total = torch.zeros(1, dtype=torch.int64).pin_memory()
        self.feat = torch.empty(3 * max_rays, dtype=torch.float32, device=device)
        self.depth = torch.empty(max_rays, dtype=torch.float32, device=device)
        self.alpha = torch.empty(max_rays, dtype=torch.float32, device=device)
        self.drop = torch.empty(max_rays, dtype=torch.float32, device=device)
        self.ev_count = torch.cuda.Event()
        self.ev_sort = torch.cuda.Event()

    def out_for(self, sensor: Sensor) -> RenderOut:
        R = sensor.n_rays
        return RenderOut(self.feat[: 3 * R].view(3, R), self.depth[:R], self.alpha[:R],
                         self.drop[:R] if sensor.is_lidar else None, None, None)


class Server:
    def __init__(self, g_cam: GaussianSet, g_lidar: GaussianSet, sensors: list, pool_bytes: int,
                 n_slots: int = 12, n_workgroups: int = 1024, params=None, abk=(1.0, 2.0, 0.0)):
        self.g_cam, self.g_lidar, self.sensors = g_cam, g_lidar, sensors
        dev = g_cam.mean.device
        self.dev = dev
        self.params = params or render_params()
        self.abk = abk
        self.n_workgroups = n_workgroups
        self.pool = DevicePool(pool_bytes, dev)
        max_rays = max(s.n_rays for s in sensors)
        self.slots = [Slot(g_cam.n, max_rays, dev) for _ in range(n_slots)]
        self.comp_streams = [torch.cuda.Stream(device=dev) for _ in range(2)]
        self.batch_ws = [torch.empty(int(lib().ut_batch_workspace_bytes(n_slots)), dtype=torch.uint8, device=dev)
                         for _ in range(2)]
        self.count_bytes = int(lib().ut_count_workspace_bytes(g_cam.n))
        self.stats = {}

    def _g(self, sensor: Sensor) -> GaussianSet:
        return self.g_lidar if sensor.is_lidar else self.g_cam

    def _start(self, r: Request):
        L = lib()
        s = r.slot
        sensor = self.sensors[r.sensor]
        g = self._g(sensor)
        st = _stream(s.stream)
        import ctypes as C
        abk = (C.c_double * 3)(*self.abk)
        gc = g.c()
        check(L.ut_project(ref(gc), ref(sensor.c), C.cast(abk, C.c_void_p), ref(s.p.c()), st), "ut_project")
        check(L.ut_bin_count(ref(s.p.c()), g.n, ref(sensor.c), s.ws.data_ptr(), s.ws.numel(), s.total.data_ptr(), st),
              "ut_bin_count")
        s.ev_count.record(s.stream)

    def _need(self, r: Request):
        sensor = self.sensors[r.sensor]
        pw = int(lib().ut_pair_workspace_bytes(r.n_pairs))
        lb = 4 * max(r.n_pairs, 1)
        rb = 8 * sensor.n_super
        return pw, lb, rb

    def _sort(self, r: Request):
        L = lib()
        s = r.slot
        sensor = self.sensors[r.sensor]
        g = self._g(sensor)
        pw, lb, rb = self._need(r)
        al = lambda v: (v + ALIGN - 1) // ALIGN * ALIGN
        pbuf = self.pool.view(r.mem, 0, pw)
        gauss = self.pool.view(r.mem, al(pw), lb).view(torch.int32)
        ranges = self.pool.view(r.mem, al(pw) + al(lb), rb).view(torch.int32).view(2, sensor.n_super)
        r.bins = BinLists(gauss, ranges, r.n_pairs)
        check(L.ut_bin_sort(ref(s.p.c()), g.n, ref(sensor.c), s.ws.data_ptr(), s.ws.numel(), pbuf.data_ptr(), pw,
                            r.n_pairs, ref(r.bins.c()), _stream(s.stream)), "ut_bin_sort")
        s.ev_sort.record(s.stream)

    def _composite(self, reqs, k):
        cs = self.comp_streams[k]
        n = len(reqs)
        arr = (A.UtBatchItem * n)()
        keep = []
        for i, r in enumerate(reqs):
            cs.wait_event(r.slot.ev_sort)
            sensor = self.sensors[r.sensor]
            r.out = r.slot.out_for(sensor)
            pc, lc, oc = r.slot.p.c(), r.bins.c(), r.out.c()
            keep += [pc, lc, oc]
            arr[i] = A.UtBatchItem(ref(pc), ref(lc), ref(sensor.c), ref(oc))
        import ctypes as C
        ws = self.batch_ws[k]
        check(lib().ut_composite_batch(C.cast(arr, C.c_void_p), n, ref(self.params), ws.data_ptr(), ws.numel(),
                                       self.n_workgroups, _stream(cs)), "ut_composite_batch")
        ev = torch.cuda.Event()
        ev.record(cs)
        return ev

    def run(self, trace, on_done=None, max_batch=None):
        """trace: list of (arrival_seconds, frame_id, sensor_index) sorted by arrival.
        on_done(request) is called (outputs still valid) before the slot is reused."""
        with _collector_paused():
            return self._run(trace, on_done, max_batch)

    def _run(self, trace, on_done, max_batch):
        reqs = [Request(i, int(f), int(si), float(t)) for i, (t, f, si) in enumerate(trace)]
        waiting, counting, counted, sorting, batches = deque(), [], deque(), [], []
        free_slots = list(self.slots)
        free_comp = [0, 1]
        n_done, i_next = 0, 0
        n_batches, batch_sizes, max_mem_wait = 0, [], 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        while n_done < len(reqs):
            t = now()
            progressed = False
            while i_next < len(reqs) and reqs[i_next].arrival <= t:
                waiting.append(reqs[i_next])
                i_next += 1
            while waiting and free_slots:
                r = waiting.popleft()
                r.slot = free_slots.pop()
                r.t_start = now()
                self._start(r)
                counting.append(r)
                progressed = True
            for r in list(counting):
                if r.slot.ev_count.query():
                    counting.remove(r)
                    r.n_pairs = int(r.slot.total.item())
                    r.t_counted = now()
                    counted.append(r)
                    progressed = True
            max_mem_wait = max(max_mem_wait, len(counted))
            while counted:
                r = counted[0]
                pw, lb, rb = self._need(r)
                al = lambda v: (v + ALIGN - 1) // ALIGN * ALIGN
                blk = self.pool.alloc(al(pw) + al(lb) + al(rb))
                if blk is None:
                    if not sorting and not batches and self.pool.in_use == 0:
                        raise RuntimeError(f"request {r.rid} needs more than the whole pool")
                    break
                counted.popleft()
                r.mem = blk
                r.t_sort = now()
                self._sort(r)
                sorting.append(r)
                progressed = True
            if sorting and free_comp:
                ready = [r for r in sorting if r.slot.ev_sort.query()]
                if max_batch:
                    ready = ready[:max_batch]
                if ready:
                    tb = now()
                    for r in ready:
                        sorting.remove(r)
                        r.t_batch = tb
                    k = free_comp.pop(0)
                    ev = self._composite(ready, k)
                    batches.append((ev, ready, k))
                    n_batches += 1
                    batch_sizes.append(len(ready))
                    progressed = True
            for item in list(batches):
                ev, rs, k = item
                if ev.query():
                    td = now()
                    for r in rs:
                        r.t_done = td
                        if on_done is not None:
                            on_done(r)
                        self.pool.release(r.mem)
                        free_slots.append(r.slot)
                    n_done += len(rs)
                    batches.remove(item)
                    free_comp.append(k)
                    progressed = True
            if not progressed:
                time.sleep(20e-6)
        stage = lambda a, b: round(float(np.mean([getattr(r, b) - getattr(r, a) for r in reqs])) * 1e3, 3)
        self.stats = {"batches": n_batches, "mean_batch": float(np.mean(batch_sizes)) if batch_sizes else 0.0,
                      "pool_peak_bytes": self.pool.peak, "max_waiting_for_memory": max_mem_wait,
                      # mean milliseconds a request spends between consecutive stages
                      "stage_ms": {"slot_wait": stage("arrival", "t_start"), "count": stage("t_start", "t_counted"),
                                   "memory_wait": stage("t_counted", "t_sort"), "sort": stage("t_sort", "t_batch"),
                                   "composite": stage("t_batch", "t_done")}}
        return reqs


def run_plain(g_cam, g_lidar, sensors, trace, pipes=None, on_done=None):
    """The same arrival trace served one request at a time, first come first served, with
    the single-request path (no overlap between requests)."""
    if pipes is None:
        pipes = [SensorPipeline(g_lidar if s.is_lidar else g_cam, s) for s in sensors]
    with _collector_paused():
        return _run_plain(pipes, trace, on_done)


def _run_plain(pipes, trace, on_done):
    reqs = [Request(i, int(f), int(si), float(t)) for i, (t, f, si) in enumerate(trace)]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        while time.perf_counter() - t0 < r.arrival:
            time.sleep(20e-6)
        pipes[r.sensor].run(stream)
        stream.synchronize()
        r.t_done = time.perf_counter() - t0
        r.n_pairs = pipes[r.sensor].n_pairs
        if on_done is not None:
            r.out = pipes[r.sensor].out
            on_done(r)
    return reqs, pipes


def poisson_trace(rate_fps: float, seconds: float, n_sensors: int, seed: int = 0):
    """Frames arrive as a Poisson process; each frame issues one request per sensor."""
    rng = np.random.default_rng(seed)
    t, f, out = 0.0, 0, []
    while True:
        t += rng.exponential(1.0 / rate_fps)
        if t > seconds:
            break
        for si in range(n_sensors):
            out.append((t, f, si))
        f += 1
    return out


def frame_latencies(reqs):
    frames = {}
    for r in reqs:
        a, d = frames.get(r.frame, (r.arrival, r.t_done))
        frames[r.frame] = (min(a, r.arrival), max(d, r.t_done))
    lat = np.array([d - a for a, d in frames.values()])
    return lat


def summarize(reqs, rays_per_request):
    lat = frame_latencies(reqs)
    rl = np.array([r.t_done - r.arrival for r in reqs])
    span = max(r.t_done for r in reqs) - min(r.arrival for r in reqs)
    rays = sum(rays_per_request[r.sensor] for r in reqs)
    return {"frames": int(len(lat)), "p50_frame_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_frame_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "p50_request_ms": round(float(np.percentile(rl, 50)) * 1e3, 3),
            "p99_request_ms": round(float(np.percentile(rl, 99)) * 1e3, 3),
            "mrays_per_s": round(rays / span / 1e6, 2)}


def bench_served(g, gl, sensors_np, sensors, dev, args, log):
    """Served vs plain on Poisson traces at 30 frames/s per simulated vehicle."""
    rays = [s.n_rays for s in sensors]
    out = {"rate_per_vehicle_fps": 30, "seconds": args.served_seconds, "vehicles": {}}
    pool_bytes = 48 << 30
    server = Server(g, gl, sensors, pool_bytes=pool_bytes, n_slots=14)
    pipes = None
    # warm both paths
    warm = poisson_trace(60.0, 0.1, len(sensors), seed=99)
    server.run(warm)
    _, pipes = run_plain(g, gl, sensors, warm, pipes)
    for v in [int(x) for x in args.vehicles.split(",") if x]:
        trace = poisson_trace(30.0 * v, args.served_seconds, len(sensors), seed=v)
        sreq = server.run(trace)
        srv = summarize(sreq, rays)
        srv.update(server.stats)
        preq, pipes = run_plain(g, gl, sensors, trace, pipes)
        pl = summarize(preq, rays)
        out["vehicles"][str(v)] = {"served": srv, "plain": pl}
        log(f"V={v}: served p50/p99 {srv['p50_frame_ms']}/{srv['p99_frame_ms']} ms {srv['mrays_per_s']} Mrays/s | "
            f"plain p50/p99 {pl['p50_frame_ms']}/{pl['p99_frame_ms']} ms {pl['mrays_per_s']} Mrays/s")
    return out
