"""Serving loop: host-side logic on the CPU (allocator, arrival process, latency maths with a
fake clock) and, on the GPU, served results bit-identical to plain renders under memory
pressure and overlap."""
import numpy as np
import pytest

from paper_2510_12901_amd import serve


def test_collector_paused_inside_a_loop_and_restored():
    import gc
    was = gc.isenabled()
    try:
        for start in (True, False):
            (gc.enable if start else gc.disable)()
            with serve._collector_paused():
                assert not gc.isenabled()
            assert gc.isenabled() == start
        gc.enable()
        with pytest.raises(ValueError):
            with serve._collector_paused():
                raise ValueError("request failed")
        assert gc.isenabled()   # restored on the error path too
    finally:
        (gc.enable if was else gc.disable)()


def test_pool_first_fit_and_merge():
    pool = serve.DevicePool(4096, device="cpu")
    a = pool.alloc(1000)          # rounds to 1024
    b = pool.alloc(1000)
    c = pool.alloc(2048)
    assert a == (0, 1024) and b == (1024, 1024) and c == (2048, 2048)
    assert pool.alloc(1) is None  # full: admission must wait
    pool.release(b)
    assert pool.alloc(2000) is None
    pool.release(a)               # merges with b's hole
    assert pool.alloc(2000) == (0, 2048)
    assert pool.peak == 4096


def test_poisson_trace_rate_and_frames():
    tr = serve.poisson_trace(240.0, 20.0, 7, seed=3)
    frames = len(tr) // 7
    assert abs(frames / 20.0 - 240.0) < 240.0 * 0.05
    assert all(tr[i][0] <= tr[i + 1][0] for i in range(len(tr) - 1))
    assert [t[2] for t in tr[:7]] == list(range(7))


def test_latency_summary_with_fake_clock():
    reqs = []
    for f in range(100):
        for s in range(2):
            reqs.append(serve.Request(len(reqs), f, s, arrival=f * 0.01, t_done=f * 0.01 + 0.002 + 0.001 * s + (0.05 if f == 99 else 0)))
    out = serve.summarize(reqs, [100, 200])
    assert out["frames"] == 100
    assert abs(out["p50_frame_ms"] - 3.0) < 1e-6
    assert out["p99_frame_ms"] > 3.0
    span = reqs[-1].t_done - reqs[0].arrival
    assert abs(out["mrays_per_s"] - 300 * 100 / span / 1e6) < 0.01


@pytest.mark.gpu
def test_served_results_bit_identical_to_plain_under_memory_pressure():
    import torch
    import paper_2510_12901_amd as ut
    import synth
    g_np, gl_np, sensors_np = synth.scene_multisensor(5, n=30000, n_cameras_pinhole=2, n_cameras_fisheye=1,
                                                      pinhole_size=(160, 96), fisheye_size=(128, 96),
                                                      lidar_beams=32, lidar_az=512)
    dev = torch.device("cuda")
    g = ut.GaussianSet.from_numpy(g_np, dev)
    gl = ut.GaussianSet(g.mean, g.quat, g.log_scale, g.opacity_logit,
                        torch.as_tensor(gl_np["feat"], device=dev), 0, synth.FEAT_LIDAR)
    sensors = [ut.Sensor(s, dev) for s in sensors_np]
    ref = []
    for s in sensors:
        _, lists, out = ut.render(gl if s.is_lidar else g, s, state=False)
        ref.append({k: getattr(out, k).cpu().numpy() for k in ("feat", "depth", "alpha")} |
                   ({"drop": out.drop.cpu().numpy()} if out.drop is not None else {}))
        ref[-1]["pairs"] = lists.n_pairs
    # a pool that holds about two requests at a time forces admission waits
    need = max(int(ut.lib().ut_pair_workspace_bytes(r["pairs"])) + 4 * r["pairs"] + 8 * s.n_tiles + 1024
               for r, s in zip(ref, sensors))
    server = serve.Server(g, gl, sensors, pool_bytes=2 * need + 4096, n_slots=4, n_workgroups=512)
    trace = serve.poisson_trace(2000.0, 0.05, len(sensors), seed=1)
    assert len(trace) >= 40
    seen = []

    def check(r):
        got = {k: getattr(r.out, k).cpu().numpy() for k in ("feat", "depth", "alpha")}
        if r.out.drop is not None:
            got["drop"] = r.out.drop.cpu().numpy()
        for k, v in got.items():
            assert np.array_equal(v, ref[r.sensor][k]), (r.rid, k)
        seen.append(r.rid)

    reqs = server.run(trace, on_done=check)
    assert sorted(seen) == list(range(len(trace)))
    assert server.stats["max_waiting_for_memory"] >= 1
    assert server.stats["pool_peak_bytes"] <= server.pool.nbytes
    assert server.stats["mean_batch"] >= 1.0
    assert all(r.t_done >= r.arrival for r in reqs)
    # every request passed the stages in order
    assert all(r.arrival <= r.t_start <= r.t_counted <= r.t_sort <= r.t_batch <= r.t_done for r in reqs)
    assert set(server.stats["stage_ms"]) == {"slot_wait", "count", "memory_wait", "sort", "composite"}
    assert server.stats["stage_ms"]["memory_wait"] > 0.0


@pytest.mark.gpu
def test_request_larger_than_pool_is_rejected():
    import torch
    import paper_2510_12901_amd as ut
    import synth
    g_np, s_np = synth.scene_pinhole_small(0)
    g = ut.GaussianSet.from_numpy(g_np)
    s = ut.Sensor(s_np)
    server = serve.Server(g, g, [s], pool_bytes=4096, n_slots=2)
    with pytest.raises(RuntimeError, match="whole pool"):
        server.run([(0.0, 0, 0)])


@pytest.mark.gpu
def test_served_thin_discs_bit_identical_to_plain():
    """The batched compositing kernel on records that take the residual form of D^2 (discs
    1e-3 to 1e-5 as thick as they are wide): every served result equals the plain render."""
    import torch
    import paper_2510_12901_amd as ut
    import synth
    rng = np.random.default_rng(8)
    n = 4000
    mean = np.stack([rng.uniform(-10, 10, n), rng.uniform(-7, 7, n), rng.uniform(15, 60, n)])
    g_np = synth.particles(rng, mean, 0.3, 1.5, 0, synth.FEAT_CAMERA)
    w = rng.uniform(np.log(0.3), np.log(1.5), n)
    g_np["log_scale"] = np.stack([w, w + rng.uniform(-0.5, 0.5, n),
                                  w + rng.uniform(np.log(1e-5), np.log(1e-3), n)]).astype(np.float32)
    g = ut.GaussianSet.from_numpy(g_np)
    sensors = [ut.Sensor(synth.pinhole(160, 120, 220.0, 220.0)), ut.Sensor(synth.pinhole(128, 96, 150.0, 150.0))]
    ref = []
    for s in sensors:
        _, _, out = ut.render(g, s, state=False)
        ref.append({k: getattr(out, k).cpu().numpy() for k in ("feat", "depth", "alpha")})
    assert (ref[0]["alpha"] > 0).mean() > 0.5
    server = serve.Server(g, g, sensors, pool_bytes=64 << 20, n_slots=4, n_workgroups=512)
    trace = serve.poisson_trace(1000.0, 0.03, len(sensors), seed=2)
    seen = []

    def check(r):
        for k in ("feat", "depth", "alpha"):
            assert np.array_equal(getattr(r.out, k).cpu().numpy(), ref[r.sensor][k]), (r.rid, k)
        seen.append(r.rid)

    server.run(trace, on_done=check)
    torch.cuda.synchronize()
    assert sorted(seen) == list(range(len(trace))) and len(seen) >= 10
