"""Benchmark: RGB+D frames/s at 256x256, batched vs per-view, with step
latency, a roofline for the dominant kernel and the CPU oracle baseline.

Workload (batch64_4scenes_256): 64 environments over 4 synthetic jittered
apartments of 100k / 250k / 500k / 1M triangles, one 256x256 RGB+D view per
environment per step, poses from per-environment random walks (0.25 m
forward moves, 10 degree turns).  A step renders the 64 views of one walk
step; inputs (scenes, poses staged by the library) are resident before the
timed region starts.

Output: one JSON line on stdout; progress on stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RGB+D frames/sec at 256x256 (batched vs per-view) ; p50/p99 step latency"
HBM_PEAK_GBS = 8000.0
# one int32/fp32 VALU lane operation per lane per clock: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# algorithmic VALU work of the raster stage: 8 ops per bbox pixel test (three
# edge functions at 2 ops, a combine, a compare) and 12 more per covered
# fragment (three int->float, four multiplies, two adds, compare/select)
RASTER_PHASES = ("raster8", "raster16", "raster32")
OPS_PER_TEST = 8
OPS_PER_COVERED = 12


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` as rocprofv3's FETCH_SIZE/WRITE_SIZE
    counted them (scaled by a plain-copy calibration), recorded by
    paper_1904_01201_amd.rocprof_summary; None if the record is for another
    kernel or the kernel sources changed since it was taken."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1904_01201_amd", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
        from paper_1904_01201_amd.rocprof_summary import source_hash
    except (OSError, ValueError, ImportError):
        return None
    if t.get("kernel") != kernel or t.get("source_sha256") != source_hash():
        return None
    return t


def other_workloads(ctx, a):
    """Throughput of the plain path on the room and apartment-walk
    workloads (one hab_render call per view, in order, one stream) and of
    the mixed 256-environment batch through the captured stepper."""
    import torch
    from scenegen import configs
    out = {}

    def plain(w, W, H):
        sc = ctx.upload_scene(w.scenes[0])
        sn = ctx.sensor(W, H)
        o = ctx.alloc(sn, 1)
        poses = w.poses[:, 0]
        for p in poses[:5]:
            ctx.render_plain(sc, sn, p, o["rgb"], o["depth"])
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for p in poses:
            t1 = time.perf_counter()
            ctx.render_plain(sc, sn, p, o["rgb"], o["depth"])
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t1)
        el = time.perf_counter() - t0
        ctx.release(sc)
        lat = np.array(lat) * 1e3
        return {"frames_per_s": round(len(poses) / el, 1), "views": int(len(poses)),
                "p50_ms": round(float(np.percentile(lat, 50)), 4),
                "p99_ms": round(float(np.percentile(lat, 99)), 4),
                "triangles": int(w.scenes[0].num_triangles), "resolution": [W, H],
                "path": "hab_render, one view per call, synchronised per view"}

    out["room_2k_128"] = plain(configs.room_2k_128(), 128, 128)
    log(f"room_2k_128 plain: {out['room_2k_128']['frames_per_s']} frames/s")
    out["apartment_200k_256"] = plain(configs.apartment_200k_256(), 256, 256)
    log(f"apartment_200k_256 plain: {out['apartment_200k_256']['frames_per_s']} frames/s")

    steps = max(10, min(a.steps, 50))
    w = configs.batch256_16scenes_mixed(steps=steps + 5)
    hs = [ctx.upload_scene(s) for s in w.scenes]
    sensors = {}
    for s in w.env_sensor:
        if (s.width, s.outputs) not in sensors:
            sensors[(s.width, s.outputs)] = ctx.sensor(s.width, s.height, s.hfov_deg, s.near_m, s.outputs)
    items = []
    for e in range(w.num_envs):
        sn = sensors[(w.env_sensor[e].width, w.env_sensor[e].outputs)]
        o = ctx.alloc(sn, 1)
        items.append((hs[w.env_scene[e]], sn, w.poses[0, e], o.get("rgb"), o.get("depth"), None))
    ctx.autotune(items)
    st = ctx.stepper(items)
    for s_ in range(5):
        st.step(w.poses[s_])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in range(steps):
        st.step(w.poses[5 + s_])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st.close()
    for h in hs:
        ctx.release(h)
    px = sum(s.width * s.height for s in w.env_sensor)
    out["batch256_16scenes_mixed"] = {
        "frames_per_s": round(w.num_envs * steps / el, 1), "ms_per_step": round(1e3 * el / steps, 4),
        "pixels_per_s": round(px * steps / el), "envs": w.num_envs, "scenes": len(w.scenes),
        "triangles": [int(s.num_triangles) for s in w.scenes], "steps": steps,
        "path": "HIP-graph stepper, autotuned", "sensors": "128/256/512 px x D/RGB/RGB+D per environment"}
    log(f"batch256_16scenes_mixed graph: {out['batch256_16scenes_mixed']['frames_per_s']} frames/s")
    return out


NAV_HEIGHTS = (0.1, 1.5)   # cross-section heights of the agent's body (just above the floor; its top)


CPU_SHARE = 16   # host CPUs per GPU on the measurement boxes


def actuation_leg(ctx, w, a, hs):
    """The agent step before rendering: batched actuation with
    collide-and-slide for 16,384 agents per scene of the bench workload
    (65,536 agents), uniformly random actions (forward twice as likely as
    each turn), timed over the bench's step count; the obstacles are the
    rendered meshes' own cross-sections (hab_nav_from_scene).  Then batched
    free-space queries: 1M random floor points per scene."""
    import torch
    from scenegen import agents_from_states
    from scenegen.walks import random_free_states
    per = 16384
    t0 = time.perf_counter()
    navs = [ctx.nav_from_scene(h, NAV_HEIGHTS) for h in hs]
    t_nav = time.perf_counter() - t0
    states, owner = [], []
    for i, s in enumerate(w.scenes):
        x, z, yaw = random_free_states(s, per, seed=500 + i)
        states.append(agents_from_states(x, z, yaw))
        owner += [i] * per
    n = per * len(w.scenes)
    ag = torch.from_numpy(np.concatenate(states)).cuda()
    rng = np.random.default_rng(3)
    steps = max(a.steps, 1)
    acts = torch.from_numpy(rng.choice([1, 1, 2, 3], size=(steps + a.warmup, n)).astype(np.uint8)).cuda()
    hit = torch.empty(n, dtype=torch.uint8, device="cuda")
    poses = torch.empty((n, 12), dtype=torch.float32, device="cuda")
    nav_of = ctx.nav_array([navs[i] for i in owner])
    for s in range(a.warmup):
        ctx.actuate(nav_of, ag, acts[s], hit, poses)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        ctx.actuate(nav_of, ag, acts[a.warmup + s], hit, poses)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # free-space queries
    nq = 1 << 20
    pts, outs = [], []
    for s in w.scenes:
        lo, hi = s.positions.min(0), s.positions.max(0)
        p = np.stack([rng.uniform(lo[0], hi[0], nq), rng.uniform(lo[2], hi[2], nq)], 1)
        pts.append(torch.from_numpy(p).cuda())
        outs.append(torch.empty(nq, dtype=torch.uint8, device="cuda"))
    for i, nv in enumerate(navs):
        ctx.nav_free(nv, pts[i], 0.1, outs[i])
    torch.cuda.synchronize()
    qsteps = max(1, min(steps, 20))
    t0 = time.perf_counter()
    for _ in range(qsteps):
        for i, nv in enumerate(navs):
            ctx.nav_free(nv, pts[i], 0.1, outs[i])
    torch.cuda.synchronize()
    el_q = time.perf_counter() - t0
    free_frac = float(np.mean([o.float().mean().item() for o in outs]))
    for nv in navs:
        ctx.nav_release(nv)
    out = {"agents": n, "scenes": len(w.scenes), "segments": [int(nv.num_segments) for nv in navs],
           "obstacles": f"mesh cross-sections at {list(NAV_HEIGHTS)} m (hab_nav_from_scene)",
           "nav_from_scene_s": round(t_nav, 4),
           "steps": steps, "agent_steps_per_s": round(n * steps / el), "ms_per_step": round(1e3 * el / steps, 4),
           "path": "hab_actuate (fp64 collide-and-slide over a uniform grid of obstacle segments, cells 0.1-0.5 m)",
           "free_space_queries_per_s": round(len(navs) * nq * qsteps / el_q),
           "free_space_query": f"hab_nav_free, {nq} random points per scene, radius 0.1 m, "
                               f"{free_frac:.2f} free"}
    log(f"actuation: {out['agent_steps_per_s']:.3g} agent steps/s ({out['ms_per_step']} ms per "
        f"{n}-agent step); free space: {out['free_space_queries_per_s']:.3g} queries/s")
    return out


def serving_leg(ctx, w, hs):
    """The serving form on the bench workload: one 256x256 RGB+D agent per
    environment (64) over the 4 resident scenes, each walking its own path;
    closed-loop saturation for 0.5 s, then Poisson arrivals at 70% of it for
    1 s (p50/p99 from arrival to completion)."""
    import paper_1904_01201_amd as P
    from paper_1904_01201_amd import loadgen
    sensor = ctx.sensor(256, 256)
    agents = loadgen.Agents(ctx, hs, w.env_scene, [sensor] * w.num_envs, w.poses)
    srv = P.Server(ctx, num_streams=3, max_batch=256)
    sat, lat_sat = loadgen.saturate(srv, agents, seconds=0.5)
    thr, lat, e2e, bs = loadgen.open_loop(srv, agents, rate=0.7 * sat, seconds=1.0, seed=7)
    st = srv.stats()
    srv.close()
    pct = lambda x, q: round(float(np.percentile(x, q)), 3) if x.size else None
    out = {"agents": w.num_envs, "saturation_rps": round(sat, 1), "offered_rps": round(0.7 * sat, 1),
           "throughput_rps": round(thr, 1), "p50_ms": pct(e2e, 50), "p99_ms": pct(e2e, 99),
           "server_p50_ms": pct(lat, 50), "server_p99_ms": pct(lat, 99),
           "mean_batch": round(float(bs.mean()), 1) if bs.size else None, "requests": int(lat.size),
           "scratch_bytes": int(st["scratch_bytes"]), "streams": 3,
           "latency": "p50/p99 arrival -> completion at 70% of closed-loop saturation; server_* submit -> completion"}
    log(f"serving: saturation {sat:.0f} requests/s, at 70%: p50 {out['p50_ms']} ms, p99 {out['p99_ms']} ms")
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measured_copy_gbs(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Device-to-device copy bandwidth (bytes read + written per second),
    timed with events on the current stream: the attainable HBM rate."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--per-view-steps", type=int, default=10)
    ap.add_argument("--latency-steps", type=int, default=100)
    ap.add_argument("--cpu-views", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="skip the room / apartment-walk / mixed-batch lines")
    ap.add_argument("--tile-size", type=int, default=0)
    ap.add_argument("--profile-only", action="store_true",
                    help="only the batched path (warmup + steps), for profiler runs")
    ap.add_argument("--one-sequence", action="store_true",
                    help="with --profile-only: render each step as one launch sequence "
                         "(every kernel alone on the GPU)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run plain 256 MiB device copies (reference for FETCH/WRITE_SIZE)")
    ap.add_argument("--serve", action="store_true",
                    help="serving curve: resident scenes, Poisson arrivals, p50/p99 vs throughput")
    ap.add_argument("--serve-agents", type=int, default=512)
    ap.add_argument("--serve-seconds", type=float, default=1.5)
    ap.add_argument("--serve-total-tri", type=int, default=20_000_000)
    ap.add_argument("--serve-scenes", type=int, default=32)
    a = ap.parse_args()
    if a.serve:
        return serve(a)
    if a.copy_calibration:
        import torch
        n = 256 << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": True, "bytes_per_copy": n, "copies": 4}), flush=True)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this renderer runs on one GPU; --gpus must be 1 "
                          "(the multi-GPU sharding is a design note only)"}))
        sys.exit(2)

    import torch
    import paper_1904_01201_amd as P
    from scenegen import configs

    t0 = time.time()
    w = configs.batch64_4scenes_256(steps=max(a.steps, a.warmup, a.latency_steps, 1))
    E = w.num_envs
    log(f"workload {w.name}: {E} envs, T={[s.num_triangles for s in w.scenes]}, "
        f"{w.num_steps} steps, generated in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    ctx = P.Context(0)
    hs = [ctx.upload_scene(s) for s in w.scenes]
    sensor = ctx.sensor(256, 256)
    out = ctx.alloc(sensor, E)
    rgb, depth = out["rgb"], out["depth"]
    items0 = [(hs[w.env_scene[e]], sensor, w.poses[0, e], rgb[e], depth[e], None) for e in range(E)]
    views = ctx.make_views(items0)
    import ctypes as C
    from paper_1904_01201_amd import binding as B

    def set_poses(step):
        ctx.set_poses(views, w.poses[step % w.num_steps])

    one_seq = a.profile_only and a.one_sequence

    def batch_step(step):
        set_poses(step)
        ctx.render_batch(None, views=views, tile_size=a.tile_size, one_sequence=one_seq)

    # ---------------------------------------------------- autotune (untimed)
    tuned = None
    if not a.tile_size:
        t0 = time.perf_counter()
        ts, bf = ctx.autotune(items0)
        tuned = {"first_class_tile": ts, "first_class_bin_factor": bf}
        log(f"autotune: tile {ts}, bin factor {bf} for the first batch class "
            f"({time.perf_counter() - t0:.2f}s)")

    # ---------------------------------------------------- batched (eager)
    for s in range(a.warmup):
        batch_step(s)
    torch.cuda.synchronize()
    # per-phase breakdown: every phase timed, over the same poses, untimed
    ctx.profile_phases(None)
    ctx.profile(True)
    for s in range(a.steps):
        batch_step(s)
    torch.cuda.synchronize()
    ctx.profile(False)
    phases = ctx.profile_read()
    # the timed steps: HIP events only around the raster launches
    ctx.profile_phases(RASTER_PHASES)
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        batch_step(s)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    ctx.profile(False)
    timed = ctx.profile_read()
    ctx.profile_phases(None)
    for k, v in timed.items():
        phases[k] = v      # the dominant kernel's time is the one taken in the timed steps
    fps_batch = E * a.steps / t_batch
    log(f"batched eager: {fps_batch:.0f} frames/s ({1e3 * t_batch / a.steps:.3f} ms/step)")
    log("phases (ms/step): " + ", ".join(f"{k}={v['ms'] / a.steps:.4f} ({v['launches'] / a.steps:g} launches)"
                                         for k, v in phases.items()))

    if a.profile_only:
        print(json.dumps({"profile_only": True, "batched_fps": round(fps_batch, 1),
                          "phase_ms_per_step": {k: v["ms"] / a.steps for k, v in phases.items()},
                          "phase_ms_per_launch": {k: v["ms"] / max(v["launches"], 1)
                                                  for k, v in phases.items()}}), flush=True)
        ctx.close()
        return

    # ---------------------------------------------------- one launch sequence
    # The same steps with the batch kept in one launch sequence (no halves
    # side by side): its rate, and the raster's duration when no other
    # kernel shares the GPU with it (reported beside the roofline).
    ctx.profile_phases(RASTER_PHASES)
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        set_poses(s)
        ctx.render_batch(None, views=views, tile_size=a.tile_size, one_sequence=True)
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    ctx.profile(False)
    one_phases = ctx.profile_read()
    ctx.profile_phases(None)
    fps_one = E * a.steps / t_one
    log(f"batched eager, one launch sequence: {fps_one:.0f} frames/s")
    # and with the atomic-free lane-owned z-test (same outputs)
    ctx.profile_phases(RASTER_PHASES)
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        set_poses(s)
        ctx.render_batch(None, views=views, tile_size=a.tile_size, one_sequence=True, lane_owned_z=True)
    torch.cuda.synchronize()
    t_lo = time.perf_counter() - t0
    ctx.profile(False)
    lo_phases = ctx.profile_read()
    ctx.profile_phases(None)
    log(f"batched eager, one launch sequence, lane-owned z-test: {E * a.steps / t_lo:.0f} frames/s")

    # ---------------------------------------------------- batched (graph)
    st = ctx.stepper(items0, tile_size=a.tile_size)
    for s in range(a.warmup):
        st.step(w.poses[s % w.num_steps])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        st.step(w.poses[s % w.num_steps])
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    fps_graph = E * a.steps / t_graph
    st.close()
    log(f"batched graph: {fps_graph:.0f} frames/s")

    # ---------------------------------------------------- env loop
    # the whole environment step on the device: actuation of the 64 agents
    # (random actions, collide-and-slide) feeding the captured render step
    from scenegen import agents_from_states
    from scenegen.walks import random_free_states
    navs_h = [ctx.nav_from_scene(h, NAV_HEIGHTS) for h in hs]
    ag_np = np.concatenate([agents_from_states(*random_free_states(w.scenes[w.env_scene[e]], 1, seed=900 + e))
                            for e in range(E)])
    ag = torch.from_numpy(ag_np).cuda()
    env_poses = torch.empty((E, 12), dtype=torch.float32, device="cuda")
    nav_of = ctx.nav_array([navs_h[w.env_scene[e]] for e in range(E)])
    # a stop action writes the starting camera poses (the library's own mapping)
    ctx.actuate(nav_of, ag, torch.zeros(E, dtype=torch.uint8, device="cuda"), None, env_poses)
    start_poses = env_poses.cpu().numpy()
    acts = torch.from_numpy(np.random.default_rng(4).choice([1, 1, 2, 3], size=(a.steps + a.warmup, E))
                            .astype(np.uint8)).cuda()
    st = ctx.stepper([(hs[w.env_scene[e]], sensor, start_poses[e], rgb[e], depth[e], None)
                      for e in range(E)], tile_size=a.tile_size)
    for s in range(a.warmup):
        ctx.actuate(nav_of, ag, acts[s], None, env_poses)
        st.step_device(env_poses)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        ctx.actuate(nav_of, ag, acts[a.warmup + s], None, env_poses)
        st.step_device(env_poses)
    torch.cuda.synchronize()
    t_env = time.perf_counter() - t0
    st.close()
    for nv in navs_h:
        ctx.nav_release(nv)
    fps_env = E * a.steps / t_env
    log(f"env loop (actuation + graph render, device poses): {fps_env:.0f} frames/s")

    # ---------------------------------------------------- per-view
    pv_steps = max(1, min(a.per_view_steps, a.steps))
    for e in range(E):
        ctx.render_plain(hs[w.env_scene[e]], sensor, w.poses[0, e], rgb[e:e + 1], depth[e:e + 1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(pv_steps):
        p = w.poses[s % w.num_steps]
        for e in range(E):
            ctx.render_plain(hs[w.env_scene[e]], sensor, p[e], rgb[e:e + 1], depth[e:e + 1])
    torch.cuda.synchronize()
    t_pv = time.perf_counter() - t0
    fps_pv = E * pv_steps / t_pv
    log(f"per-view: {fps_pv:.0f} frames/s")

    # ---------------------------------------------------- step latency
    lat = []
    for s in range(a.latency_steps):
        t0 = time.perf_counter()
        batch_step(s)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    lat_ms = np.array(lat) * 1e3
    p50, p99 = float(np.percentile(lat_ms, 50)), float(np.percentile(lat_ms, 99))
    log(f"step latency p50 {p50:.3f} ms, p99 {p99:.3f} ms")

    # ---------------------------------------------------- sensor variants
    # the same batch with the semantic instance mask written beside RGB+D,
    # with noisy depth (sigma 0.1 / m, a fresh seed per view and step), and
    # with the scenes textured (2048^2 RGB textures, 256 texels per metre)
    def variant_fps(sn, sem=None, noisy=False, handles=None):
        hv = hs if handles is None else handles
        items_v = [(hv[w.env_scene[e]], sn, w.poses[0, e], rgb[e], depth[e], None,
                    None if sem is None else sem[e], e) for e in range(E)]
        views_v = ctx.make_views(items_v)
        if not a.tile_size:
            ctx.autotune(items_v)      # its own batch class (the output mix is part of the key)

        def step_v(step):
            ctx.set_poses(views_v, w.poses[step % w.num_steps])
            if noisy:
                for e in range(E):
                    views_v[e].noise_seed = (step << 16) | e
            ctx.render_batch(None, views=views_v, tile_size=a.tile_size)

        for s in range(a.warmup):
            step_v(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(a.steps):
            step_v(s)
        torch.cuda.synchronize()
        return E * a.steps / (time.perf_counter() - t0)

    sem = torch.empty((E, 256, 256), dtype=torch.int32, device="cuda")
    fps_sem = variant_fps(ctx.sensor(256, 256, 90.0, 0.01, P.OUT_RGB | P.OUT_DEPTH | P.OUT_SEMANTIC), sem)
    del sem
    log(f"batched eager, RGB + depth + semantic: {fps_sem:.0f} frames/s")
    fps_noisy = variant_fps(ctx.sensor(256, 256, depth_noise_sigma=0.1), noisy=True)
    log(f"batched eager, RGB + noisy depth: {fps_noisy:.0f} frames/s")
    from scenegen import with_texture
    hs_tex = [ctx.upload_scene(with_texture(s)) for s in w.scenes]
    fps_tex = variant_fps(sensor, handles=hs_tex)
    for h in hs_tex:
        ctx.release(h)
    log(f"batched eager, textured RGB + depth: {fps_tex:.0f} frames/s")

    # ---------------------------------------------------- work counters
    # the same poses as the timed steps, rendered again with counters on
    bbox_tests = covered = survivors = 0
    for s_ in range(a.steps):
        set_poses(s_)
        stats = ctx.render_batch(None, views=views, tile_size=a.tile_size, stats=True)
        bbox_tests += sum(x["bbox_tests"] for x in stats)
        covered += sum(x["covered"] for x in stats)
        survivors += sum(x["survivors"] for x in stats)
    bbox_tests //= a.steps
    covered //= a.steps
    survivors //= a.steps
    assert ctx.get_error() == 0

    # ---------------------------------------------------- roofline
    # A step of 32 views or more is two launch sequences (halves of the
    # batch) that run side by side: per-launch times are each half's own
    # kernel durations, and the work of one launch is half a step's.
    per_launch = {k: v["ms"] / max(v["launches"], 1) for k, v in phases.items()}
    per_step = {k: v["ms"] / a.steps for k, v in phases.items()}
    lps = {k: v["launches"] / a.steps for k, v in phases.items()}
    raster = [k for k in phases if k.startswith("raster")]
    if raster:
        # every raster launch of a launch sequence (one per tile size in use) together
        per_launch["raster"] = sum(phases[k]["ms"] for k in raster) / max(phases[raster[0]]["launches"], 1)
        per_step["raster"] = sum(phases[k]["ms"] for k in raster) / a.steps
        lps["raster"] = lps[raster[0]]
    dom = max(((k, v) for k, v in per_launch.items() if k not in raster), key=lambda kv: kv[1])[0]
    geom_bytes = sum(15 * s.num_vertices + 12 * s.num_triangles for s in w.scenes)
    out_bytes = E * 256 * 256 * 7
    step_bytes = out_bytes + geom_bytes + 48 * E
    if dom == "raster":
        ops = (OPS_PER_TEST * bbox_tests + OPS_PER_COVERED * covered) / lps[dom]
        ach = ops / (per_launch[dom] * 1e-3) / 1e12
        # the default raster form: balanced steps (k_raster<TS, false>)
        kern = "+".join(f"k_raster<{k[6:]}, false>" for k in raster)
        tr = measured_traffic(kern)
        roof = {"kernel": kern, "bound": "alu", "achieved": round(ach, 4),
                "peak": round(ALU_PEAK_TOPS, 2), "unit": "TOP/s", "frac": round(ach / ALU_PEAK_TOPS, 5),
                "traffic": round(tr["bytes_per_launch"]) if tr else None,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "avg_launch_ms": round(per_launch[dom], 5),
                "launches_per_step": lps[dom],
                "work_per_launch": {"bbox_tests": round(bbox_tests / lps[dom]),
                                    "covered": round(covered / lps[dom]), "ops": round(ops)}}
        ms_one = sum(one_phases[k]["ms"] for k in raster if k in one_phases) / a.steps
        ops_one = OPS_PER_TEST * bbox_tests + OPS_PER_COVERED * covered
        roof_one = {"kernel": kern, "what": "the same steps in one launch sequence: one raster "
                    "launch per step with no other kernel beside it (not the timed steps)",
                    "achieved": round(ops_one / (ms_one * 1e-3) / 1e12, 4), "unit": "TOP/s",
                    "frac": round(ops_one / (ms_one * 1e-3) / 1e12 / ALU_PEAK_TOPS, 5),
                    "avg_launch_ms": round(ms_one, 5), "fps": round(fps_one, 1),
                    "lane_owned_z": {"avg_launch_ms": round(sum(lo_phases[k]["ms"] for k in raster
                                                                if k in lo_phases) / a.steps, 5),
                                     "fps": round(E * a.steps / t_lo, 1)}}
    else:
        roof_one = None
        byts = (geom_bytes + E * 16 * 8 if dom == "setup" else step_bytes) / lps[dom]
        ach = byts / (per_launch[dom] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None,
                "avg_launch_ms": round(per_launch[dom], 5)}
    ms_step = 1e3 * t_batch / a.steps
    copy_gbs = measured_copy_gbs()
    hbm = {"algorithmic_bytes_per_step": step_bytes,
           "achieved_GBs": round(step_bytes / (ms_step * 1e-3) / 1e9, 2),
           "peak_GBs": HBM_PEAK_GBS,
           "frac": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
           "measured_copy_GBs": round(copy_gbs, 1),
           "frac_of_measured_copy": round(step_bytes / (ms_step * 1e-3) / 1e9 / copy_gbs, 5)}
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")

    # ---------------------------------------------------- the other workloads
    others = {} if a.no_other_workloads else other_workloads(ctx, a)
    actuation = actuation_leg(ctx, w, a, hs)
    serving = serving_leg(ctx, w, hs)

    # ---------------------------------------------------- CPU oracle baseline
    cpu = None
    if not a.no_cpu_baseline and a.cpu_views > 0:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        # the host's share for one GPU is 16 CPUs (a pool sized to the
        # visible count could oversubscribe it); the count visible is reported
        threads = max(1, min(CPU_SHARE, os.cpu_count() or 1))
        jobs = []
        for k in range(a.cpu_views):
            s_, e_ = divmod(k, E)
            jobs.append((w.env_scene[e_], w.poses[s_ % w.num_steps, e_]))
        log(f"cpu oracle: {len(jobs)} views on {threads} threads ...")

        def one(job):
            si, pose = job
            sc = w.scenes[si]
            oracle.render_view(sc.positions, sc.colors, sc.indices, 256, 256, pose)

        t0, c0 = time.perf_counter(), time.process_time()
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(one, jobs))
        t_cpu, c_cpu = time.perf_counter() - t0, time.process_time() - c0
        n1 = min(len(jobs), E)
        t0 = time.perf_counter()
        for job in jobs[:n1]:
            one(job)
        t_one = time.perf_counter() - t0
        cpu = {"value": round(len(jobs) / t_cpu, 2), "unit": "frames/s", "cores": threads,
               "kind": "oracle",
               "sample": f"first {len(jobs)} views (steps 0..{(len(jobs) - 1) // E}) of the same "
                         f"workload, one view per thread, {t_cpu:.1f}s wall, {c_cpu:.1f} CPU-s",
               "single_thread_value": round(n1 / t_one, 2),
               "single_thread_sample": f"first {n1} views (step 0), one thread, {t_one:.1f}s",
               "host_cpus_visible": os.cpu_count(), "cpu_share_used": threads,
               "cpu_model": cpu_model()}
        log(f"cpu oracle: {cpu['value']} frames/s")
        # the two plain-path workloads, timed in full on the same threads
        full = {}
        for name, wl, px in (("room_2k_128", configs.room_2k_128(), 128),
                             ("apartment_200k_256", configs.apartment_200k_256(), 256)):
            sc = wl.scenes[0]
            views = wl.poses[:, 0]

            def one_full(pose, sc=sc, px=px):
                oracle.render_view(sc.positions, sc.colors, sc.indices, px, px, pose)

            t0 = time.perf_counter()
            with ThreadPoolExecutor(max_workers=threads) as ex:
                list(ex.map(one_full, views))
            el = time.perf_counter() - t0
            full[name] = {"frames_per_s": round(len(views) / el, 2), "views": len(views),
                          "threads": threads, "wall_s": round(el, 2)}
            log(f"cpu oracle {name}: {full[name]['frames_per_s']} frames/s ({len(views)} views)")
        cpu["full_workloads"] = full

    res = {
        "metric": METRIC,
        "value": round(fps_batch, 1),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "envs": E, "scenes": len(w.scenes),
                   "triangles": [s.num_triangles for s in w.scenes], "resolution": [256, 256],
                   "outputs": "rgb+depth", "hfov_deg": 90.0, "path": "hab_render_batch",
                   "tile_size": a.tile_size or "autotuned", "autotune": tuned},
        "batched_fps": round(fps_batch, 1),
        "batched_graph_fps": round(fps_graph, 1),
        "env_loop_fps": round(fps_env, 1),
        "batched_rgbd_semantic_fps": round(fps_sem, 1),
        "batched_rgb_noisy_depth_fps": round(fps_noisy, 1),
        "batched_textured_rgbd_fps": round(fps_tex, 1),
        "per_view_fps": round(fps_pv, 1),
        "batched_over_per_view": round(fps_batch / fps_pv, 2),
        "p50_step_ms": round(p50, 4),
        "p99_step_ms": round(p99, 4),
        "phase_ms_per_step": {k: round(v, 5) for k, v in per_step.items()},
        "phase_ms_per_launch": {k: round(v, 5) for k, v in per_launch.items()},
        "launches_per_step": lps.get("raster", 1),
        "work": {"survivors": survivors, "bbox_tests": bbox_tests, "covered": covered},
        "roofline": roof,
        "roofline_one_sequence": roof_one,
        "hbm_roofline": hbm,
        "cpu_baseline": cpu,
        "other_workloads": others,
        "actuation": actuation,
        "serving": serving,
        "paper_context": {"rgbd_256_fps_1proc": 1042, "rgbd_256_fps_5proc": 1774,
                          "hardware": "Titan Xp + Xeon E5-2690 v4, OpenGL, Matterport3D scene"},
    }
    print(json.dumps(res), flush=True)
    ctx.close()


def serve(a):
    """Serving curve on the serve_32scenes workload (32 resident jittered
    apartments, sum T ~ 20M, agents with mixed 128/256/512 resolutions and
    D/RGB/RGB+D sensors)."""
    import torch
    import paper_1904_01201_amd as P
    from paper_1904_01201_amd import loadgen
    from scenegen import configs

    t0 = time.time()
    w = configs.serve_32scenes(num_agents=a.serve_agents, steps=64, total_T=a.serve_total_tri,
                               num_scenes=a.serve_scenes)
    log(f"serve workload: {len(w.scenes)} scenes, sum T = {sum(s.num_triangles for s in w.scenes)}, "
        f"{w.num_envs} agents, generated in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    ctx = P.Context(0)
    hs = [ctx.upload_scene(s) for s in w.scenes]
    resident = sum(h.device_bytes for h in hs)
    sensors = [ctx.sensor(s.width, s.height, s.hfov_deg, s.near_m, s.outputs) for s in w.env_sensor]
    agents = loadgen.Agents(ctx, hs, w.env_scene, sensors, w.poses)
    srv = P.Server(ctx, num_streams=3, max_batch=256)
    # closed loop at 1, 2, 4, ... agents (each keeps one request in flight)
    agents_curve = []
    na = 1
    while na <= w.num_envs:
        thr, lat_c = loadgen.saturate(srv, agents, seconds=min(a.serve_seconds, 0.5), num=na)
        agents_curve.append({"agents": na, "throughput_rps": round(thr, 1),
                             "p50_ms": round(float(np.percentile(lat_c, 50)), 3),
                             "p99_ms": round(float(np.percentile(lat_c, 99)), 3), "requests": int(lat_c.size)})
        log(f"closed loop, {na} agents: {agents_curve[-1]}")
        na *= 2
    sat, lat_sat = loadgen.saturate(srv, agents, seconds=a.serve_seconds)
    log(f"closed-loop saturation ({w.num_envs} agents): {sat:.0f} requests/s, "
        f"p50 {np.percentile(lat_sat, 50):.2f} ms")
    # open loop: Poisson arrivals from 10% to 120% of saturation, at least
    # 10k requests per point
    curve = []
    for frac in (0.1, 0.3, 0.5, 0.7, 0.9, 1.1, 1.2):
        rate = frac * sat
        secs = min(10.0, max(a.serve_seconds, 10_000 / rate))
        thr, lat, e2e, bs = loadgen.open_loop(srv, agents, rate=rate, seconds=secs, seed=int(frac * 100))
        pct = lambda x, q: round(float(np.percentile(x, q)), 3) if x.size else None
        pt = {"offered_frac": frac, "offered_rps": round(rate, 1), "throughput_rps": round(thr, 1),
              "p50_ms": pct(e2e, 50), "p99_ms": pct(e2e, 99),
              "server_p50_ms": pct(lat, 50), "server_p99_ms": pct(lat, 99),
              "mean_batch": round(float(bs.mean()), 1) if bs.size else None, "requests": int(lat.size),
              "seconds": round(secs, 2)}
        curve.append(pt)
        log(f"offered {frac:.1f}x: {pt}")
    st = srv.stats()
    srv.close()
    assert ctx.get_error() == 0
    ctx.close()
    px = [s.width * s.height for s in w.env_sensor]
    print(json.dumps({"metric": "serving: step-request latency p50/p99 vs throughput",
                      "unit": "requests/s", "saturation_rps": round(sat, 1),
                      "config": {"workload": w.name, "scenes": len(w.scenes),
                                 "total_triangles": int(sum(s.num_triangles for s in w.scenes)),
                                 "resident_bytes": int(resident), "agents": w.num_envs,
                                 "mean_pixels_per_request": round(float(np.mean(px)), 1),
                                 "streams": 3, "max_batch": 256},
                      "latency": "p50/p99 arrival -> completion; server_* submit -> completion",
                      "agents_curve": agents_curve, "curve": curve, "server_stats": st}), flush=True)


if __name__ == "__main__":
    main()
