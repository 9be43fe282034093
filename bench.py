#!/usr/bin/env python3
"""Benchmark of the UT Gaussian rasterizer on one MI355X.

Workload (the multi-sensor simulation frame): 2,000,000 particles resident in HBM, one frame
= 4 pinhole cameras 1920x1080 + 2 fisheye cameras 1920x1280 + 1 spinning LiDAR 128x2048
(13,471,744 rays).  A timed step renders one frame through the whole hot path for every
sensor: sigma-point projection (+ LiDAR ray culling), depth and super-tile radix sorts,
compositing (with on-chip per-tile list compaction).  Inputs are seeded and synthetic and
already resident when timing starts.  Prints ONE JSON line: the frame throughput, the
compositing kernel against its float64 roofline, the oracle timed on the host, and the
adjoint, time-dependent, beam-divergence, actor and serving measurements beside them.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

# Hardware queues of this process, set before the HIP runtime starts: the frame's 7 sensor
# streams each get a queue of their own instead of sharing the runtime's default 4 (measured:
# 3.44 -> 3.52-3.56 Grays/s); far more queues oversubscribe the scheduler (32 halved the
# served throughput).  --hw-queues overrides it.
def _hw_queues_from_argv(default: int = 8) -> str:
    for i, a in enumerate(sys.argv):
        if a == "--hw-queues" and i + 1 < len(sys.argv):
            return sys.argv[i + 1]
        if a.startswith("--hw-queues="):
            return a.split("=", 1)[1]
    return str(default)


os.environ["GPU_MAX_HW_QUEUES"] = _hw_queues_from_argv()

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6        # MI355X dense float64 vector (FMA = 2 FLOPs)
PEAK_HBM_GBS = 8000.0
# float64 FLOPs (FMA = 2) of the compositing's work, counted from the arithmetic of the
# method in the record's quadric form: every (ray, list entry) pair a ray evaluates needs
# d^T B d from the ray's six monomials (11), d^T B v (5), num = v^T B v d^T B d - (d^T B v)^2
# (3), the cut (2) and the pre-test num > cut d^T B d (1); a pair that passes the pre-test adds
# 1/d^T B d with two Newton steps (9), t* (1), D^2 = max(num, 0) / d^T B d (2), the exponent
# (1), exp (17), alpha = min(sigma rho, alpha_max) (2), w = alpha T (1), 4 accumulations (8)
# and T (1 - alpha) (2).  The kernel counts both kinds of pair per ray (n_visit, n_pass) in an
# untimed pass; entries dropped by the tile-cone test are never evaluated and not counted.
FLOPS_PER_VISIT = 22
SETUP_FRAMES = 8
FLOPS_PER_PASS = 43
# The compositing roof in VALU lane-operations: every (ray, particle) pair a ray evaluates is
# priced at the method's 65 lane-ops (compensated cross product 21, N c 9, |.|^2 3, M d 9,
# |M d|^2 3, t* 3, reciprocal 2, exp 2, alpha 3, weight / transmittance / accumulators 8,
# tests 2), against 256 CUs x 64 float64 (= non-packed float32) lanes per clock x 2.4 GHz.
# The adjoint prices a replayed pair at 2.5 times the forward's work.
LANE_OPS_PER_PAIR = 65
ADJOINT_LANE_OPS_PER_PAIR = 162.5
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12     # 39.3 T lane-ops/s
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "composite_traffic.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("composite.hip", "ut_cone.hpp", "ut_internal.hpp", "ut_device.hpp"):   # the kernel and its headers
        h.update(open(os.path.join(ROOT, "paper_2510_12901_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--particles", type=int, default=2_000_000)
    ap.add_argument("--streams", type=int, default=7, help="HIP streams the sensors of a frame are spread over")
    ap.add_argument("--hw-queues", type=int, default=8,
                    help="hardware queues of the process (GPU_MAX_HW_QUEUES, set before the runtime starts)")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-time-dependent", action="store_true")
    ap.add_argument("--no-beam-divergence", action="store_true")
    ap.add_argument("--no-actors", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the per-configuration stage timings")
    ap.add_argument("--no-spatial-order", action="store_true",
                    help="keep the multi-sensor scene in generation order instead of Z-order")
    ap.add_argument("--host-count", action="store_true",
                    help="read each sensor's pair total on the host before sorting (one mid-frame sync)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--served-seconds", type=float, default=10.0, help="measured seconds of arrivals per trace")
    ap.add_argument("--served-warmup", type=float, default=1.0, help="warm-up seconds of arrivals per trace")
    ap.add_argument("--vehicles", type=str, default="1,2,4,6,8,12,16")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 1 GiB device copy (reference kernel for HBM counters)")
    ap.add_argument("--lidar-sweep", action="store_true",
                    help="instead of the frame benchmark: LiDAR tiling sweep (N_phi x M) and culling ablation "
                         "on the 300,000-particle 128x2048 LiDAR workload")
    ap.add_argument("--config-only", type=int, choices=(0, 1, 2, 3), default=None,
                    help="instead of the frame benchmark: render one single-sensor workload (0: pinhole "
                         "128x96, 1: fisheye 1920x1280, 2: LiDAR 128x2048, 3: pinhole 1920x1080) K times with the "
                         "pair total kept on the GPU, for a kernel profile of that workload alone")
    ap.add_argument("--summarize-profiles", nargs=3, metavar=("STATS_CSV", "FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/ summaries from rocprofv3 CSV output (kernel stats, FETCH_SIZE "
                         "and WRITE_SIZE counter collections) instead of benchmarking")
    return ap.parse_args()


CAMERA_KERNEL = "k_composite<256, 1, 128, false, false>"
PROFILE_CMDS = {
    "stats": "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_stats -o kt -- "
             "python -u bench.py --no-served --no-backward --no-cpu-baseline --no-time-dependent --no-beam-divergence "
             "--no-actors --no-configs --steps 5 --warmup 1 --streams 1",
    "fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch -o f -- "
             "python -u bench.py --no-served --no-backward --no-cpu-baseline --no-time-dependent --no-beam-divergence "
             "--no-actors --no-configs --steps 2 --warmup 1 --streams 1 --calib-copy",
    "write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_write -o w -- "
             "python -u bench.py --no-served --no-backward --no-cpu-baseline --no-time-dependent --no-beam-divergence "
             "--no-actors --no-configs --steps 2 --warmup 1 --streams 1 --calib-copy",
}


def _short_kernel(name: str) -> str:
    import re
    m = re.search(r"(k_\w+(<[^>]*>)?|__amd_\w+|\w+_kernel\w*)", name)
    return m.group(1) if m else name[:40]


def summarize_profiles(stats_csv: str, fetch_csv: str, write_csv: str):
    """Turn rocprofv3 CSV output into profiles/*.md and profiles/composite_traffic.json.

    HBM traffic of the camera compositing kernel: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) averaged over its dispatches, each scaled by the factor that makes the same
    counter read exactly 1 GiB for the 1 GiB device copy of --calib-copy."""
    import csv

    stats = list(csv.DictReader(open(stats_csv)))
    lines = ["# Kernel time, multisensor frame (2M particles, 7 sensors, one stream)", "",
             "Command (from the repository root, on the GPU):", "", "    cd /tmp && export TMPDIR=/tmp  # then, in the repo:",
             "    " + PROFILE_CMDS["stats"], "",
             "The run covers 1 warm-up + 5 timed frames, the 5 back-to-back compositing launches per camera "
             "that bench.py times for the roofline, and one state pass.", "",
             "| kernel | calls | avg us | min us | max us | % of GPU time |", "|---|---|---|---|---|---|"]
    for r in stats[:20]:
        lines.append(f"| `{_short_kernel(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    cam = [r for r in stats if CAMERA_KERNEL in r["Name"]]
    cam_avg_us = float(cam[0]["AverageNs"]) / 1e3 if cam else None
    lines += ["", f"`{CAMERA_KERNEL}` (camera compositing) average: {cam_avg_us:.1f} us over "
              f"{cam[0]['Calls'] if cam else 0} calls."]
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    open(os.path.join(ROOT, "profiles", "kernels_multisensor_frame.md"), "w").write("\n".join(lines) + "\n")

    def counter(path, cname):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == cname]
        comp = [float(r["Counter_Value"]) for r in rows if CAMERA_KERNEL in r["Kernel_Name"]]
        copies = [(int(r["Grid_Size"]), float(r["Counter_Value"])) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        ref_kib = max(copies)[1]              # the largest copy is the 1 GiB reference
        factor = (1 << 20) / ref_kib          # KiB that 1 GiB should read as / KiB measured
        return float(np.mean(comp)), len(comp), ref_kib, factor

    f_kib, nf, f_ref, f_fac = counter(fetch_csv, "FETCH_SIZE")
    w_kib, nw, w_ref, w_fac = counter(write_csv, "WRITE_SIZE")
    fetch_b = f_kib * 1024 * f_fac
    write_b = w_kib * 1024 * w_fac
    traffic = {"kernel": CAMERA_KERNEL, "workload": "multisensor", "kernel_source_hash": kernel_source_hash(),
               "bytes_per_launch": round(fetch_b + write_b), "fetch_bytes": round(fetch_b), "write_bytes": round(write_b),
               "fetch_kib_raw": round(f_kib, 1), "write_kib_raw": round(w_kib, 1), "dispatches": [nf, nw],
               "calibration": {"copy_bytes": 1 << 30, "fetch_kib_read": f_ref, "write_kib_read": w_ref,
                               "fetch_factor": round(f_fac, 4), "write_factor": round(w_fac, 4)}}
    json.dump(traffic, open(PROFILE_TRAFFIC, "w"), indent=1)
    md = ["# HBM traffic of the camera compositing kernel (multisensor frame)", "",
          "Commands (two separate counter passes; from the repository root on the GPU, TMPDIR=/tmp):", "",
          "    " + PROFILE_CMDS["fetch"], "    " + PROFILE_CMDS["write"], "",
          f"Averaged over {nf} / {nw} dispatches of `{CAMERA_KERNEL}` (the 6 cameras equally).", "",
          "| counter | raw KiB per dispatch | 1 GiB copy reads as (KiB) | factor | bytes per launch |",
          "|---|---|---|---|---|",
          f"| FETCH_SIZE | {f_kib:.1f} | {f_ref:.1f} | {f_fac:.4f} | {fetch_b / 1e6:.1f} MB |",
          f"| WRITE_SIZE | {w_kib:.1f} | {w_ref:.1f} | {w_fac:.4f} | {write_b / 1e6:.1f} MB |", "",
          f"Traffic per launch: {(fetch_b + write_b) / 1e6:.1f} MB (kernel source hash {traffic['kernel_source_hash']}, "
          "over composite.hip and the headers it includes; "
          "bench.py reports it only while the hash matches)."]
    open(os.path.join(ROOT, "profiles", "composite_traffic_multisensor.md"), "w").write("\n".join(md) + "\n")
    print(json.dumps(traffic))


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


CONFIG_SCENES = ("scene_pinhole_small", "scene_fisheye", "scene_lidar", "scene_pinhole_large")


def config_only(args):
    """One single-sensor workload alone: W warm-up renders, then K renders with the pair total
    kept on the GPU (each synchronised); prints the median frame time."""
    import torch

    import paper_2510_12901_amd as ut
    import synth

    dev = torch.device("cuda:0")
    g_np, s_np = getattr(synth, CONFIG_SCENES[args.config_only])(args.seed)
    g = ut.GaussianSet.from_numpy(g_np, dev)
    s = ut.Sensor(s_np, dev)
    pipe = ut.SensorPipeline(g, s)
    stream = torch.cuda.current_stream()
    for _ in range(SETUP_FRAMES + args.warmup):
        pipe.run(stream)
    torch.cuda.synchronize()
    pipe.set_capacity(int(pipe.n_pairs * 1.25) + 4096)
    pipe.run_device(stream)
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        pipe.run_device(stream)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    if pipe.overflowed():
        raise RuntimeError("pair capacity exceeded")
    print(json.dumps({"workload": CONFIG_SCENES[args.config_only], "rays": s.n_rays, "bin_pairs": pipe.n_pairs,
                      "frame_ms_device_count": round(float(np.median(times)) * 1e3, 4)}))


def lidar_sweep(args):
    """Tiling sweep and culling ablation on the LiDAR workload (300,000 particles, 128 beams x
    2048 azimuth steps): for every (N_phi, M) the whole LiDAR render (projection with culling,
    binning, sort, compositing) is timed frame by frame over K frames after W warm-up frames
    (median), and the compositing alone over 5 back-to-back launches."""
    import torch

    import paper_2510_12901_amd as ut
    import synth

    dev = torch.device("cuda:0")
    g_np, s0 = synth.scene_lidar(args.seed, n=300_000)
    g = ut.GaussianSet.from_numpy(g_np, dev)
    beams = s0["beam_elev"]
    stream = torch.cuda.current_stream()

    def time_config(n_phi, M, cull):
        s = ut.Sensor(synth.lidar(beams, 2048, n_phi=n_phi, max_per_tile=M, cull=cull), dev)
        pipe = ut.SensorPipeline(g, s)
        for _ in range(SETUP_FRAMES + args.warmup):
            pipe.run(stream)
        torch.cuda.synchronize()
        times = []     # per-frame wall time, median: robust to a one-off host stall in a launch
        for _ in range(args.steps):
            t0 = time.perf_counter()
            pipe.run(stream)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        frame_ms = float(np.median(times)) * 1e3
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            pipe.composite_only(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return {"n_phi": n_phi, "M": M, "cull": cull, "n_theta": int(s.c.n_theta),
                "max_tile_rays": s.max_tile_rays, "bin_pairs": pipe.n_pairs, "frame_ms": round(frame_ms, 4),
                "mrays_per_s": round(s.n_rays / frame_ms / 1e3, 2),
                "composite_ms": round(e0.elapsed_time(e1) / 5, 4)}

    rows = []
    for n_phi in (64, 32, 16, 8):
        for M in (256, 128, 64, 32):
            r = time_config(n_phi, M, True)
            rows.append(r)
            log(json.dumps(r))
    abl = [time_config(16, 32, c) for c in (True, False)]
    for r in abl:
        log(json.dumps(r))
    print(json.dumps({"lidar_tiling_sweep": rows, "culling_ablation": abl}))


def main():
    args = parse()
    if args.summarize_profiles:
        summarize_profiles(*args.summarize_profiles)
        return
    if args.lidar_sweep:
        lidar_sweep(args)
        return
    if args.config_only is not None:
        config_only(args)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the rasterizer has no multi-GPU path in this build", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2510_12901_amd as ut
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        a.fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    t_setup = time.time()
    g_np, gl_np, sensors_np = synth.scene_multisensor(args.seed, n=args.particles)
    g = ut.GaussianSet.from_numpy(g_np, dev)
    gl = ut.GaussianSet(g.mean, g.quat, g.log_scale, g.opacity_logit,
                        torch.as_tensor(gl_np["feat"], device=dev), 0, synth.FEAT_LIDAR)
    if not args.no_spatial_order:
        # the resident scene is stored along the Z-order curve of the means (once, at upload;
        # images do not depend on the order, the projection's reads do)
        perm = ut.spatial_order(g)
        g = ut.gather(g, perm)
        gl_feat = ut.gather(gl, perm).feat
        gl = ut.GaussianSet(g.mean, g.quat, g.log_scale, g.opacity_logit, gl_feat, 0, synth.FEAT_LIDAR)
        torch.cuda.synchronize()
        del perm
    sensors = [ut.Sensor(s, dev) for s in sensors_np]
    pipes = [ut.SensorPipeline(gl if s.is_lidar else g, s) for s in sensors]
    rays_per_frame = sum(s.n_rays for s in sensors)
    log(f"setup {time.time() - t_setup:.1f}s, rays/frame {rays_per_frame}")

    stream = torch.cuda.current_stream()
    # the sensors of a frame are independent: spread them over a few streams (default
    # priority) so that one sensor's small binning kernels overlap another's compositing
    streams = [torch.cuda.Stream(device=dev) for _ in range(min(args.streams, len(pipes)))]
    torch.cuda.synchronize()

    device_count = False

    def frame(events=None):
        if device_count:
            # the pair totals stay on the GPU: each sensor's whole render is enqueued on its
            # stream at once (capacities from the set-up frames; overflow checked afterwards)
            for i, p in enumerate(pipes):
                st = streams[i % len(streams)]
                p.project_and_count(st)
                p.sort_and_composite_device(st, None if events is None else events[i])
            return
        # every sensor's projection + pair count first, one host synchronisation for the
        # seven pair totals, then every sensor's sort + compositing
        for i, p in enumerate(pipes):
            p.project_and_count(streams[i % len(streams)])
        for st in streams:
            st.synchronize()
        for i, p in enumerate(pipes):
            p.sort_and_composite(streams[i % len(streams)], None if events is None else events[i])

    # Setup: the HIP runtime blocks one launch for ~30 ms within the first few frames of a
    # process (measured: frame 4 of a cold start, independent of how many kernels were launched
    # before), so the pipelines are primed with SETUP_FRAMES untimed frames before the warm-up.
    for _ in range(SETUP_FRAMES):
        frame()
    torch.cuda.synchronize()
    if not args.host_count:
        for p in pipes:
            p.set_capacity(int(p.n_pairs * 1.25) + 4096)
            p.clear_overflow()
        device_count = True
    for _ in range(args.warmup):
        frame()
    torch.cuda.synchronize()
    log("warmup done")

    # ------------------------------------------------------------------ timed plain frames
    K = args.steps
    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in pipes]
          for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        frame(ev[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / K
    if any(p.overflowed() for p in pipes):
        raise RuntimeError("a sensor's pair total exceeded its capacity: frames incomplete")
    value = rays_per_frame * K / (t1 - t0) / 1e6
    comp_ms = np.array([[e[0].elapsed_time(e[1]) for e in evk] for evk in ev])   # [K, sensors]
    log(f"plain frame {ms_per_step:.2f} ms, {value:.1f} Mrays/s")

    # Dominant kernel: camera compositing (k_composite on 16x16 tiles).  Its average launch duration is
    # taken from HIP events on the rendering stream around REPS back-to-back launches per
    # camera (the queue stays full, so host launch latency is excluded); its work is the
    # visited list entries of the same launches (per-ray n_proc of an identical launch).
    REPS = 5
    cams = [p for p in pipes if not p.sensor.is_lidar]
    cam_ms, visits, passes, positions = [], 0, 0, 0
    for p in cams:
        o = ut.alloc_out(p.sensor, dev, state=True, counters=True)
        p.composite_only(stream, o)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(REPS):
            p.composite_only(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        cam_ms.append(e0.elapsed_time(e1) / REPS)
        visits += int(o.n_visit.to(torch.int64).sum().item())
        passes += int(o.n_pass.to(torch.int64).sum().item())
        positions += int(o.n_proc.to(torch.int64).sum().item())
        del o
    per_launch_ms = float(np.mean(cam_ms))
    flops_per_launch = (visits * FLOPS_PER_VISIT + passes * FLOPS_PER_PASS) / len(cams)
    achieved_flops = flops_per_launch / (per_launch_ms * 1e-3) / 1e12
    lane_ops_per_launch = LANE_OPS_PER_PAIR * visits / len(cams)
    achieved = lane_ops_per_launch / (per_launch_ms * 1e-3) / 1e12
    bin_pairs = [p.n_pairs for p in pipes]
    tile_pairs = [int(p.p.count[: p.g.n].to(torch.int64).sum().item()) for p in pipes]

    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        prof = json.load(open(PROFILE_TRAFFIC))
        if prof.get("kernel_source_hash") == kernel_source_hash() and prof.get("workload") == "multisensor":
            traffic = prof.get("bytes_per_launch")

    result = {
        "metric": "Mrays/s rendered (camera+LiDAR) and served p50/p99 frame latency vs plain",
        "value": round(value, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "setup_frames": SETUP_FRAMES,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "multisensor frame: 2,000,000 particles (SH degree 3 colour + LiDAR features), "
                               "4 pinhole 1920x1080 + 2 fisheye 1920x1280 + 1 LiDAR 128x2048",
                   "particles": args.particles, "rays_per_frame": rays_per_frame, "seed": args.seed,
                   "resident_order": "generation" if args.no_spatial_order else "z-order of the means",
                   "hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"]),
                   "tile_pairs_per_sensor": tile_pairs, "bin_pairs_per_sensor": bin_pairs},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TOPS, 2),
                     "unit": "T VALU lane-ops/s", "frac": round(achieved / PEAK_VALU_TOPS, 4), "traffic": traffic,
                     "kernel": CAMERA_KERNEL + " (camera compositing)",
                     "lane_ops_per_pair": LANE_OPS_PER_PAIR,
                     "evaluated_pairs_per_launch": int(visits / len(cams)),
                     "passes_per_launch": int(passes / len(cams)),
                     "list_positions_per_launch": int(positions / len(cams)),
                     "avg_launch_ms": round(per_launch_ms, 4),
                     "flop_model": {"flops_per_visit": FLOPS_PER_VISIT, "flops_per_pass": FLOPS_PER_PASS,
                                    "achieved_tflops": round(achieved_flops, 3), "peak_fp64_tflops": PEAK_FP64_TFLOPS,
                                    "frac": round(achieved_flops / PEAK_FP64_TFLOPS, 4)},
                     "hbm_frac": (round(traffic / (per_launch_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
                                  if traffic else None)},
        "rooflines": frame_rooflines(ut, pipes, stream, dev),
        "composite_ms_per_camera": [round(float(x), 4) for x in cam_ms],
    }

    if not args.no_backward:
        result["backward"] = bench_backward(ut, synth, dev, args)
    if not args.no_configs:
        result["configs"] = bench_configs(ut, synth, dev, args)
    if not args.no_time_dependent:
        result["time_dependent"] = bench_time_dependent(ut, synth, dev, args)
    if not args.no_beam_divergence:
        result["beam_divergence"] = bench_beam_divergence(ut, synth, dev, args)
    if not args.no_actors:
        result["actors"] = bench_actors(ut, synth, dev, args, args.particles, log)
    if not args.no_served:
        from paper_2510_12901_amd import serve
        result["served"] = serve.bench_served(g, gl, sensors_np, sensors, dev, args, log)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(g_np, gl_np, sensors_np, log)
    print(json.dumps(result), flush=True)


def _launch_ms(stream, fn, reps=5):
    """Average duration of fn() over reps back-to-back launches, HIP events on ``stream``."""
    import torch
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def frame_rooflines(ut, pipes, stream, dev):
    """The frame's other hot kernels against their roofs: LiDAR compositing (VALU lane-ops of
    its evaluated pairs) and the projection of one pinhole camera and of the LiDAR (HBM: 76 B
    per particle in and out of every particle, plus 12 K + 128 B per particle that reaches a
    tile -- its K SH coefficients per channel read, its record written)."""
    import torch
    out = {}
    lid = [p for p in pipes if p.sensor.is_lidar][0]
    o = ut.alloc_out(lid.sensor, dev, state=True, counters=True)
    lid.composite_only(stream, o)
    ms = _launch_ms(stream, lambda: lid.composite_only(stream))
    vis = int(o.n_visit.to(torch.int64).sum().item())
    a = LANE_OPS_PER_PAIR * vis / (ms * 1e-3) / 1e12
    out["lidar_composite"] = {"bound": "alu", "achieved": round(a, 3), "peak": round(PEAK_VALU_TOPS, 2),
                              "unit": "T VALU lane-ops/s", "frac": round(a / PEAK_VALU_TOPS, 4),
                              "evaluated_pairs_per_launch": vis, "avg_launch_ms": round(ms, 4),
                              "max_tile_rays": lid.sensor.max_tile_rays}
    del o
    for name, p in (("project_pinhole", [q for q in pipes if q.sensor.kind == 0][0]), ("project_lidar", lid)):
        ms = _launch_ms(stream, lambda: p.project(stream))
        n = p.g.n
        K = (p.g.sh_degree + 1) ** 2
        V = int((p.p.count[:n] > 0).sum().item())
        b = 76 * n + (12 * K + int(ut.lib().ut_record_bytes())) * V
        gbps = b / (ms * 1e-3) / 1e9
        out[name] = {"bound": "hbm", "achieved": round(gbps, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(gbps / PEAK_HBM_GBS, 4), "bytes_per_launch": b, "particles": n,
                     "reaching_a_tile": V, "avg_launch_ms": round(ms, 4)}
    return out


def bench_backward(ut, synth, dev, args):
    """Forward + adjoint of the 1,000,000-particle pinhole 1920x1080 scene with the L1 upstream."""
    import torch
    g_np, s_np = synth.scene_pinhole_large(args.seed)
    g = ut.GaussianSet.from_numpy(g_np, dev)
    s = ut.Sensor(s_np, dev)
    target = torch.as_tensor(synth.l1_target(7, (3, s.n_rays)), device=dev)
    pipe = ut.SensorPipeline(g, s, state=True)

    def step():
        out = pipe.run()
        up = torch.sign(out.feat - target) / out.feat.numel()
        return ut.backward(g, pipe.p, pipe.bins, s, out, up_feat=up)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    n = 5
    t0 = time.perf_counter()
    for _ in range(n):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / n
    # the adjoint call alone (accumulator fill, k_backward, chain rule) against the VALU roof,
    # pricing every pair the forward evaluated at the adjoint's lane-ops per pair
    stream = torch.cuda.current_stream()
    out = pipe.run()
    up = torch.sign(out.feat - target) / out.feat.numel()
    o = ut.alloc_out(s, dev, state=True, counters=True)
    pipe.composite_only(stream, o)
    vis = int(o.n_visit.to(torch.int64).sum().item())
    del o
    bms = _launch_ms(stream, lambda: ut.backward(g, pipe.p, pipe.bins, s, out, up_feat=up))
    a = ADJOINT_LANE_OPS_PER_PAIR * vis / (bms * 1e-3) / 1e12
    return {"workload": "1,000,000 particles, pinhole 1920x1080, forward + adjoint of mean L1",
            "ms_per_step": round(ms, 3), "mrays_per_s": round(s.n_rays / ms / 1e3, 2), "pairs": pipe.n_pairs,
            "roofline": {"bound": "alu", "kernel": "ut_composite_backward (fill, k_backward, k_chain)",
                         "achieved": round(a, 3), "peak": round(PEAK_VALU_TOPS, 2), "unit": "T VALU lane-ops/s",
                         "frac": round(a / PEAK_VALU_TOPS, 4), "lane_ops_per_pair": ADJOINT_LANE_OPS_PER_PAIR,
                         "forward_evaluated_pairs": vis, "avg_call_ms": round(bms, 4)}}


def _time_sensor(ut, g, d, dev, args, stream):
    """Frame time of one sensor render (projection, binning, sort, compositing; median of K
    frames after the set-up and W warm-up frames), the compositing time alone and the work
    counters of one frame."""
    import torch
    s = ut.Sensor(d, dev)
    pipe = ut.SensorPipeline(g, s)
    for _ in range(SETUP_FRAMES + args.warmup):
        pipe.run(stream)
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        pipe.run(stream)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ms = float(np.median(times)) * 1e3
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        pipe.composite_only(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    o = ut.alloc_out(s, dev, state=True, counters=True)
    pipe.composite_only(stream, o)
    torch.cuda.synchronize()
    return {"ms_per_frame": round(ms, 3), "mrays_per_s": round(s.n_rays / ms / 1e3, 2),
            "composite_ms": round(e0.elapsed_time(e1) / 5, 4), "bin_pairs": pipe.n_pairs,
            "evaluated_pairs": int(o.n_visit.to(torch.int64).sum().item()),
            "list_positions": int(o.n_proc.to(torch.int64).sum().item())}


def bench_beam_divergence(ut, synth, dev, args):
    """The 300,000-particle 128x2048 LiDAR without and with a 3 mrad beam-divergence cone
    (the smoothing widens every particle across the beam, so tiles receive more pairs)."""
    import torch
    stream = torch.cuda.current_stream()
    g_np, lid = synth.scene_lidar(args.seed)
    g = ut.GaussianSet.from_numpy(g_np, dev)
    row = {}
    for label, theta in (("off", 0.0), ("3mrad", 0.003)):
        d = dict(lid)
        d["beam_divergence"] = theta
        row[label] = _time_sensor(ut, g, d, dev, args, stream)
    log(f"beam divergence lidar_128x2048_300k: {json.dumps(row)}")
    return {"lidar_128x2048_300k": row}


def bench_actors(ut, synth, dev, args, n_particles, log):
    """The multisensor frame with a scene graph: the last 100,032 of the 2,000,000 particles
    form 64 car-sized actors (1,563 particles each, object frames, yaw poses on the ground),
    transformed to the world once per frame (ut_actor_transform) before the 7 sensors render.
    Reports the transform kernel against HBM (60 algorithmic bytes per particle: actor id,
    mean and quaternion in; mean and quaternion out), its adjoint, and the frame with and
    without the transform."""
    import torch
    n_act, per = 64, 1563
    g_np, gl_np, sensors_np = synth.scene_multisensor(args.seed, n=n_particles)
    n_bg = n_particles - n_act * per
    rng = np.random.default_rng(args.seed + 17)
    g_obj, ids, poses = synth.actors(rng, synth.subset(g_np, np.arange(n_bg)), n_act, per,
                                     [[-40, 40], [-40, 40], [-4, -3]], up_axis=2)
    lid_feat = np.concatenate([gl_np["feat"][:, :, :n_bg], synth.lidar_feat(rng, n_act * per)], 2)
    g = ut.GaussianSet.from_numpy(g_obj, dev)
    actor = torch.as_tensor(ids, device=dev)
    P = ut.actor_poses(poses).to(dev)
    lfeat = torch.as_tensor(lid_feat, device=dev)
    stream = torch.cuda.current_stream()
    gw = ut.actor_transform(g, actor, P)
    glw = ut.GaussianSet(gw.mean, gw.quat, gw.log_scale, gw.opacity_logit, lfeat, 0, synth.FEAT_LIDAR)
    sensors = [ut.Sensor(s, dev) for s in sensors_np]
    pipes = [ut.SensorPipeline(glw if s.is_lidar else gw, s) for s in sensors]

    def transform():
        ut.actor_transform(g, actor, P, out=gw, stream=stream)   # into the world set the pipelines read

    def frame(with_transform):
        if with_transform:
            transform()
        for p in pipes:
            p.project_and_count(stream)
        stream.synchronize()
        for p in pipes:
            p.sort_and_composite(stream)

    reps = 50
    for _ in range(5):
        transform()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        transform()
    e1.record(stream)
    torch.cuda.synchronize()
    t_us = e0.elapsed_time(e1) / reps * 1e3
    gmw = torch.randn_like(g.mean)
    gqw = torch.randn_like(g.quat)
    ut.actor_transform_backward(g, actor, P, gmw, gqw)
    e0.record(stream)
    for _ in range(reps):
        ut.actor_transform_backward(g, actor, P, gmw, gqw)
    e1.record(stream)
    torch.cuda.synchronize()
    b_us = e0.elapsed_time(e1) / reps * 1e3
    row = {}
    for label, wt in (("with_transform", True), ("pre_transformed", False)):
        for _ in range(SETUP_FRAMES + args.warmup):
            frame(wt)
        torch.cuda.synchronize()
        times = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            frame(wt)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        row[label + "_ms"] = round(float(np.median(times)) * 1e3, 3)
    n = g.n
    n_obj = n_act * per
    fwd_bytes = 60 * n
    # adjoint: id, world gradients in, object gradients out for every particle (60 B); the
    # object-frame mean and quaternion are read for actor particles only (+28 B)
    bwd_bytes = 60 * n + 28 * n_obj
    res = {"workload": f"{n:,} particles, {n_act} actors x {per} particles; multisensor frame (7 sensors, one stream)",
           "transform_us": round(t_us, 2), "transform_gbps": round(fwd_bytes / t_us / 1e3, 1),
           "transform_frac_hbm": round(fwd_bytes / t_us / 1e3 / PEAK_HBM_GBS, 3),
           "backward_us": round(b_us, 2), "backward_gbps": round(bwd_bytes / b_us / 1e3, 1),
           "backward_frac_hbm": round(bwd_bytes / b_us / 1e3 / PEAK_HBM_GBS, 3),
           "bytes_per_particle": {"forward": 60, "backward": "60 (background), 88 (actor)"}, **row}
    log(f"actors: {json.dumps(res)}")
    return res


def bench_configs(ut, synth, dev, args):
    """Each single-sensor workload on its own (plain path, one stream): frame time (median of K
    renders with the pair total kept on the GPU, as the multi-sensor frame renders; and with
    the host-count path's round trip) and per-stage GPU time from HIP events around projection,
    depth sort + pair count, pair emission + super-tile sort, and compositing (median of K,
    pair totals kept on the GPU so the stages run back to back).  Projection and binning are
    priced against HBM with their algorithmic bytes:
      projection: 76 B per particle (11 floats in; rects, packed rect, key, count out) plus
                  12 K + 128 B per particle that reaches a tile (K SH coefficients per channel
                  in, the record out);
      depth sort: per visible particle 4 radix passes of 16 B (key and value in and out) plus
                  4 B for the digit histogram, and 16 B per particle for the compaction;
      pair sort:  per super-tile pair 8 B emitted, 16 B per radix pass, 4 B for the ranges.
    Compositing is priced against the VALU roof (65 lane-ops per evaluated pair, counted by a
    counting launch, over the average of back-to-back launches).
    The same workloads drawn with the next two seeds are timed as whole frames (pair total kept
    on the GPU)."""
    import torch
    stream = torch.cuda.current_stream()
    K = args.steps
    cases_by_seed = {"cfg0 pinhole 128x96, 1,000 particles": synth.scene_pinhole_small,
                     "cfg1 fisheye 1920x1280, 500,000 particles": synth.scene_fisheye,
                     "cfg2 LiDAR 128x2048, 300,000 particles": synth.scene_lidar,
                     "cfg3 pinhole 1920x1080, 1,000,000 particles": synth.scene_pinhole_large}
    rows = {}
    for name, gen in cases_by_seed.items():
        g_np, s_np = gen(args.seed)
        g = ut.GaussianSet.from_numpy(g_np, dev)
        s = ut.Sensor(s_np, dev)
        pipe = ut.SensorPipeline(g, s)
        for _ in range(SETUP_FRAMES + args.warmup):
            pipe.run(stream)
        torch.cuda.synchronize()
        times = []
        for _ in range(K):
            t0 = time.perf_counter()
            pipe.run(stream)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        frame_ms = float(np.median(times)) * 1e3
        P = pipe.n_pairs
        V = int((pipe.p.count > 0).sum().item())
        pipe.set_capacity(int(P * 1.25) + 4096)
        pipe.clear_overflow()
        st_ms = {k: [] for k in ("project", "depth_sort", "pair_sort", "composite")}
        for _ in range(K):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
            ev[0].record(stream)
            pipe.project(stream)
            ev[1].record(stream)
            pipe.count(stream)
            ev[2].record(stream)
            pipe.sort_device(stream)
            ev[3].record(stream)
            pipe.composite_only(stream)
            ev[4].record(stream)
            torch.cuda.synchronize()
            for i, k in enumerate(st_ms):
                st_ms[k].append(ev[i].elapsed_time(ev[i + 1]))
        # the whole render with the pair total kept on the GPU (no host round trip inside the
        # frame, as in the multi-sensor benchmark): wall time per frame, median of K
        dtimes = []
        for _ in range(K):
            t0 = time.perf_counter()
            pipe.run_device(stream)
            torch.cuda.synchronize()
            dtimes.append(time.perf_counter() - t0)
        frame_dev_ms = float(np.median(dtimes)) * 1e3
        if pipe.overflowed():
            raise RuntimeError(f"{name}: pair capacity exceeded")
        # the compositing kernel against the VALU roof: lane-ops of the pairs it evaluates (a
        # counting launch) over the average of back-to-back launches
        oc = ut.alloc_out(s, dev, state=True, counters=True)
        pipe.composite_only(stream, oc)
        c_ms = _launch_ms(stream, lambda: pipe.composite_only(stream))
        c_vis = int(oc.n_visit.to(torch.int64).sum().item())
        del oc
        c_ach = LANE_OPS_PER_PAIR * c_vis / (c_ms * 1e-3) / 1e12
        med = {k: float(np.median(v)) for k, v in st_ms.items()}
        n, Kc = g.n, (g.sh_degree + 1) ** 2
        n_super = int(s.n_super)
        pair_passes = (max(int(np.ceil(np.log2(max(n_super, 2)))), 1) + 7) // 8
        b_proj = 76 * n + (12 * Kc + int(ut.lib().ut_record_bytes())) * V
        b_depth = 16 * n + (4 * 16 + 4) * V
        b_pair = (8 + 16 * pair_passes + 4) * P
        gbps = lambda b, ms: b / (ms * 1e-3) / 1e9
        # the primary frame keeps the pair total on the GPU (the production path, as in the
        # multi-sensor benchmark); the host-count path adds one host round trip per frame
        rows[name] = {
            "rays": s.n_rays, "frame_ms": round(frame_dev_ms, 4), "mrays_per_s": round(s.n_rays / frame_dev_ms / 1e3, 2),
            "frames_per_s": round(1e3 / frame_dev_ms, 1),
            "frame_ms_host_count": round(frame_ms, 4),
            "mrays_per_s_host_count": round(s.n_rays / frame_ms / 1e3, 2), "visible": V, "bin_pairs": P,
            "stage_ms": {k: round(v, 4) for k, v in med.items()},
            "composite_roofline": {"bound": "alu", "achieved": round(c_ach, 3), "peak": round(PEAK_VALU_TOPS, 2),
                                   "unit": "T VALU lane-ops/s", "frac": round(c_ach / PEAK_VALU_TOPS, 4),
                                   "evaluated_pairs_per_launch": c_vis, "avg_launch_ms": round(c_ms, 4)},
            "hbm_frac": {"project": round(gbps(b_proj, med["project"]) / PEAK_HBM_GBS, 3),
                         "depth_sort": round(gbps(b_depth, med["depth_sort"]) / PEAK_HBM_GBS, 3),
                         "pair_sort": round(gbps(b_pair, med["pair_sort"]) / PEAK_HBM_GBS, 3)}}
        del pipe, s, g
        # the same workload drawn with the next two seeds: frame time only
        fr = [rows[name]["frame_ms"]]
        for sd in (args.seed + 1, args.seed + 2):
            g2_np, s2_np = cases_by_seed[name](sd)
            g2 = ut.GaussianSet.from_numpy(g2_np, dev)
            s2 = ut.Sensor(s2_np, dev)
            pipe2 = ut.SensorPipeline(g2, s2)
            for _ in range(SETUP_FRAMES + args.warmup):
                pipe2.run(stream)
            torch.cuda.synchronize()
            pipe2.set_capacity(int(pipe2.n_pairs * 1.25) + 4096)
            pipe2.clear_overflow()
            ts = []
            for _ in range(K):
                t0 = time.perf_counter()
                pipe2.run_device(stream)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            if pipe2.overflowed():
                raise RuntimeError(f"{name}, seed {sd}: pair capacity exceeded")
            fr.append(round(float(np.median(ts)) * 1e3, 4))
            del pipe2, s2, g2
        rows[name]["seeds"] = {"seed": [args.seed, args.seed + 1, args.seed + 2], "frame_ms": fr,
                               "mrays_per_s": [round(rows[name]["rays"] / f / 1e3, 2) for f in fr]}
        log(f"{name}: {json.dumps(rows[name])}")
    return rows


def bench_time_dependent(ut, synth, dev, args):
    """Static vs moving sensors on the 1,000,000-particle pinhole 1920x1080 scene (rolling
    shutter: 0.5 m sideways and 0.01 rad of yaw during the readout, a side camera of a car at
    15 m/s filming at 30 frames/s) and the 300,000-particle 128x2048 LiDAR (1.5 m and 0.03 rad over one sweep,
    15 m/s at 10 Hz).  Each render (projection, binning, sort, compositing) is timed frame by
    frame (median of K after W warm-up frames)."""
    import torch
    stream = torch.cuda.current_stream()
    out = {}
    cam_g, cam = synth.scene_pinhole_large(args.seed)
    lid_g, lid = synth.scene_lidar(args.seed)
    turn = np.array([[np.cos(0.01), 0.0, -np.sin(0.01)], [0.0, 1.0, 0.0], [np.sin(0.01), 0.0, np.cos(0.01)]])
    R_cam1 = (turn @ np.asarray(cam["R_sw"], np.float64)).astype(np.float32)   # 0.01 rad about camera y
    cam_m = synth.rolling_shutter(cam, R_cam1, np.asarray(cam["origin"], np.float32) + np.array([0.5, 0, 0], np.float32))
    lid_m = synth.spinning(lid, synth.yaw_lidar_pose(0.03), np.array([1.5, 0.0, 0.0], np.float32))
    for name, g_np, descs in (("pinhole_1920x1080_1M", cam_g, (cam, cam_m)), ("lidar_128x2048_300k", lid_g, (lid, lid_m))):
        g = ut.GaussianSet.from_numpy(g_np, dev)
        row = {}
        for label, d in zip(("static", "moving"), descs):
            row[label] = _time_sensor(ut, g, d, dev, args, stream)
        out[name] = row
        log(f"time-dependent {name}: {json.dumps(row)}")
    return out


def cpu_baseline(g_np, gl_np, sensors_np, log, seed=0):
    """The oracle (FP64, OpenMP over rays/tiles) on bounded samples:
    - value: the frame's LiDAR rendered in full and one pinhole camera with every 8th ray
      composited (its projection and binning in full), all host threads;
    - one_core: the frame's LiDAR with every 4th ray composited (projection and binning in
      full) on one thread;
    - configs: the single-sensor workloads on all threads -- the 1,000-particle pinhole, the
      500,000-particle fisheye and the 300,000-particle LiDAR as full frames, the
      1,000,000-particle pinhole with every 16th ray composited, and the adjoint on the
      2,000-particle 64x64 copy of the latter (forward + backward)."""
    import oracle
    import synth
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    lid = [s for s in sensors_np if s["kind"] == 2][0]
    cam = [s for s in sensors_np if s["kind"] == 0][0]
    rays = 0
    og_l = oracle.OracleGaussians(gl_np)
    os_l = oracle.OracleSensor(lid)
    _, _, out = oracle.render(og_l, os_l)
    rays += os_l.n_rays
    og_c = oracle.OracleGaussians(g_np)
    os_c = oracle.OracleSensor(cam)
    pr = oracle.project(og_c, os_c)
    lists = oracle.bin_pairs(os_c, pr["rect"], pr["count"], pr["key"])
    ids = np.arange(0, os_c.n_rays, 8)
    oracle.composite_rays(og_c, os_c, lists, ids)
    rays += len(ids)
    dt = time.perf_counter() - t0
    del lists, pr
    log(f"cpu baseline {dt:.1f}s for {rays} rays on {threads} threads")

    def sampled(og, osn, step):
        t = time.perf_counter()
        p = oracle.project(og, osn)
        ls = oracle.bin_pairs(osn, p["rect"], p["count"], p["key"])
        sel = np.arange(0, osn.n_rays, step)
        oracle.composite_rays(og, osn, ls, sel)
        return len(sel), time.perf_counter() - t

    oracle.set_num_threads(1)
    try:
        r1, t1 = sampled(og_l, os_l, 4)
    finally:
        oracle.set_num_threads(threads)
    log(f"cpu baseline one core {t1:.1f}s for {r1} rays")

    cfg = {}
    for name, (gq, sq), step in (("cfg0 pinhole 128x96, 1,000 particles", synth.scene_pinhole_small(seed), 1),
                                 ("cfg2 LiDAR 128x2048, 300,000 particles", synth.scene_lidar(seed), 1),
                                 ("cfg1 fisheye 1920x1280, 500,000 particles", synth.scene_fisheye(seed), 1),
                                 ("cfg3 pinhole 1920x1080, 1,000,000 particles", synth.scene_pinhole_large(seed), 16)):
        og, osn = oracle.OracleGaussians(gq), oracle.OracleSensor(sq)
        if step == 1:
            t = time.perf_counter()
            oracle.render(og, osn)
            r, tt = osn.n_rays, time.perf_counter() - t
        else:
            r, tt = sampled(og, osn, step)
        cfg[name] = {"mrays_per_s": round(r / tt / 1e6, 4), "rays": r, "seconds": round(tt, 3),
                     "sample": "full frame" if step == 1 else f"every {step}th ray (projection and binning in full)"}
    gq, sq = synth.scene_pinhole_large(seed, n=2000, width=64, height=64, f=40.0)
    t = time.perf_counter()
    op, ol, oo = oracle.render(gq, sq)
    target = synth.l1_target(7, (3, 64 * 64)).astype(np.float64)
    oracle.backward(gq, sq, ol, {"feat": np.sign(oo["feat"] - target) / (3 * 64 * 64)})
    tt = time.perf_counter() - t
    cfg["cfg3 adjoint copy: 2,000 particles, 64x64, forward + backward"] = {
        "mrays_per_s": round(64 * 64 / tt / 1e6, 4), "rays": 64 * 64, "seconds": round(tt, 3), "sample": "full frame"}
    log(f"cpu baseline configs: {json.dumps(cfg)}")
    return {"value": round(rays / dt / 1e6, 4), "unit": "Mrays/s", "cores": threads,
            "kind": "oracle",
            "sample": "2,000,000-particle frame: LiDAR 128x2048 in full + pinhole 1920x1080 every 8th ray "
                      "(projection and binning in full)", "seconds": round(dt, 2), "rays": rays,
            "one_core": {"value": round(r1 / t1 / 1e6, 4), "unit": "Mrays/s", "cores": 1, "seconds": round(t1, 2),
                         "sample": "the frame's LiDAR, every 4th ray composited (projection and binning in full)"},
            "configs": cfg}


if __name__ == "__main__":
    main()
