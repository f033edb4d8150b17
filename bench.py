#!/usr/bin/env python3
"""Throughput of the sparse-local-field ray-casting renderer on one MI355X.

One step = one 1920x1080 pinhole camera frame plus one 64 x 2,048 rolling-shutter LiDAR sweep
(10 m/s) rendered from the ~2M-voxel driving scene (5 levels, 1.6 m to 0.1 m), S = 4 samples per
voxel, t_min = 1e-6.  The scene is resident in HBM before timing; ray generation is fused into the
render kernels.  Prints one JSON line:
  value      camera + LiDAR rays per second (Mrays/s) over the timed steps
  roofline   the camera render kernel (the dominant kernel): algorithmic bytes per launch
             (128 B per shaded voxel hit: density + RGB corner records, plus 20 B of outputs per
             ray) over its average duration, against the 8 TB/s HBM peak
  cpu_baseline  the CPU oracle on a bounded sample of the same rays, over a process pool
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import itertools
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CAM_HIT_BYTES, CAM_RAY_BYTES = 128, 20     # sigma + RGB corner logits (32 floats); rgb, depth, opacity
LID_HIT_BYTES, LID_RAY_BYTES = 64, 12      # sigma + intensity corner logits (16 floats); depth, intensity, opacity
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_render_multi_driving.json")
CAMERA_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_render_camera_driving.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2507_18713_amd", "csrc", f)
                  for f in ("device.hpp", "shade.hpp", "render.hip")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(launch_rays: int, path: str = TRAFFIC_FILE):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or None when the counters
    were taken on other kernel sources or another workload."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash() or t.get("rays_per_launch") != launch_rays:
        return None
    return t.get("hbm_bytes_per_launch")


# ------------------------------------------------------------------ CPU baseline (oracle)
_W = {}


def _worker_init():
    import oracle
    import synth
    _W["c0"] = oracle.prepare(synth.config0_scene())
    _W["c1"] = oracle.prepare(synth.config1_scene())


def _worker_render(args):
    import oracle
    which, o, d = args
    t0 = time.perf_counter()
    oracle.render_rays(_W[which], o, d, oracle.RenderOpts(samples=4, t_min=1e-6))
    return time.perf_counter() - t0


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_sample=1024, seed=5):
    """The oracle's rays/s on the host: all 3,072 rays of the tiny scene's camera, and seeded
    1,024-ray samples of the driving camera frame and of the LiDAR sweep against all ~2M voxels,
    each timed on its own over a process pool.  The pool uses every core this process may run on,
    up to 16 (the host CPU share of one GPU); the count, the host's total and the CPU model are
    recorded.  `value` is the camera + LiDAR sample's rate, the unit of the GPU figure."""
    import multiprocessing as mp

    import numpy as np

    import oracle
    import synth
    rng = np.random.default_rng(seed)
    legs = {}
    o0, d0, _, _ = oracle.sensor_rays(synth.config0_camera())
    legs["tiny"] = ("c0", o0.astype(np.float32), d0.astype(np.float32))
    for name, sensor in (("camera", synth.config1_camera()), ("lidar", synth.config2_lidar())):
        o, d, _, _ = oracle.sensor_rays(sensor)
        idx = rng.choice(o.shape[0], n_sample, replace=False)
        legs[name] = ("c1", o[idx].astype(np.float32), d[idx].astype(np.float32))
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    workers = max(1, min(16, allowed))
    ctx = mp.get_context("spawn")
    rates = {}
    with ctx.Pool(workers, initializer=_worker_init) as pool:
        pool.map(_worker_render, [("c0", o0[:1].astype(np.float32), d0[:1].astype(np.float32))] * workers)
        for name, (which, o, d) in legs.items():
            chunks = [(which, o[i::workers * 4], d[i::workers * 4]) for i in range(workers * 4)]
            t0 = time.perf_counter()
            cpu_s = sum(pool.map(_worker_render, chunks))
            wall = time.perf_counter() - t0
            rates[name] = {"rays": int(o.shape[0]), "wall_s": round(wall, 2), "cpu_s": round(cpu_s, 1),
                           "mrays_s": o.shape[0] / wall / 1e6}
    both = (rates["camera"]["rays"] + rates["lidar"]["rays"]) / (rates["camera"]["wall_s"] + rates["lidar"]["wall_s"])
    for r in rates.values():
        r["mrays_s"] = float(f"{r['mrays_s']:.3g}")
    return {"value": float(f"{both / 1e6:.3g}"), "unit": "Mrays/s", "cores": workers, "kind": "oracle",
            "sample": f"{n_sample} pixels of the 1920x1080 camera and {n_sample} rays of the LiDAR sweep "
                      f"(seed {seed}) against all voxels of the driving scene, timed separately; value = "
                      f"both samples' rays over their summed wall time",
            "legs": rates, "host_cpu_count": os.cpu_count(), "cores_allowed": allowed, "cpu_model": _cpu_model(),
            "note": "pool capped at 16 workers, the host CPU share of one GPU"}


# ------------------------------------------------------------------ serving (vehicle sensor rigs)
def vehicle_tick(rng, scene_index):
    """One vehicle tick: 6 pinholes 1920x1080 (HFOV 70, yaw 0, +-60, +-120, 180) and 2 equidistant
    fisheyes 1280x960 (190 deg, yaw +-90), each with a 30 us/row rolling shutter, and 2 spinning
    LiDARs (roof at 1.9 m, front bumper at 0.7 m), at a random pose on the road moving at 10 m/s."""
    import numpy as np

    import synth
    x = rng.uniform(-80.0, 80.0)
    lane = rng.choice([-1.75, 1.75])
    heading = 0.0 if rng.random() < 0.5 else 180.0
    c, s = math.cos(math.radians(heading)), math.sin(math.radians(heading))
    v = (10.0 * c, 10.0 * s, 0.0)
    frames = []
    for yaw in (0.0, 60.0, -60.0, 120.0, -120.0, 180.0):
        frames.append(("camera", synth.pinhole(1920, 1080, 70.0, synth.yaw_pitch_camera(heading + yaw, -3.0),
                                               (x, lane, 1.6), dt_line=30e-6, v=v)))
    for yaw in (90.0, -90.0):
        frames.append(("fisheye", synth.fisheye_equidistant(1280, 960, 190.0, synth.yaw_pitch_camera(heading + yaw, 0.0),
                                                            (x, lane, 1.5), dt_line=30e-6, v=v)))
    for z, dx in ((1.9, 0.0), (0.7, 2.0)):
        frames.append(("lidar", synth.lidar_spinning(64, 2048, -25.0, 15.0, synth.yaw_lidar(heading),
                                                     (x + dx * c, lane + dx * s, z), 0.1, v=v)))
    return [(kind, sen, scene_index) for kind, sen in frames]


OUTS = {"camera": ("rgb", "depth", "opacity"), "fisheye": ("rgb", "depth", "opacity"),
        "lidar": ("depth", "intensity", "opacity")}
FISHEYE_VALID = 1101128  # rays inside the 190 deg circle of a 1280x960 equidistant fisheye


def frame_rays(kind, sen):
    return FISHEYE_VALID if kind == "fisheye" else sen["width"] * sen["height"]


# server configurations (max_batch, max_inflight, max_launch_rays): launches capped at one full-HD
# frame of rays, four in flight, so that a request completes with a launch of about its own size;
# and whole admitted batches, two in flight
SERVER_CONFIGS = {"served": (32, 4, 1920 * 1080), "served_whole_batches": (32, 2, 0)}


def serving_bench(salf, torch, dev, n_ticks=500, warm_ticks=10, seed=7, pool_gib=1.0, configs=None):
    """Poisson arrivals of vehicle ticks over 4 resident scenes: plain FIFO rendering (one frame at
    a time on one stream) against the continuous-batching server, at 0.5x, 0.9x and 1.5x the plain
    capacity and in a closed loop (all ticks queued at once).  Latency = arrival to completion on
    the host monotonic clock, per frame."""
    configs = SERVER_CONFIGS if configs is None else configs
    import numpy as np

    import synth
    scenes = [salf.Scene.from_data(synth.config1_variant(s), device=dev, preactivate=True) for s in (11, 12, 13, 14)]
    rng = np.random.default_rng(seed)
    ticks = [vehicle_tick(rng, int(rng.integers(0, 4))) for _ in range(n_ticks + warm_ticks)]
    opts = dict(samples=4, t_min=1e-6)

    def plain_run(arrivals):
        # a single worker renders queued frames in arrival order, one at a time
        done, q = [], collections.deque()
        t0 = time.monotonic()
        i = 0
        frames = [(arrivals[k], f) for k, tk in enumerate(ticks) for f in tk]
        while len(done) < len(frames):
            now = time.monotonic() - t0
            while i < len(frames) and frames[i][0] <= now:
                q.append(frames[i])
                i += 1
            if not q:
                time.sleep(max(0.0, frames[i][0] - now))
                continue
            arr, (kind, sen, si) = q.popleft()
            salf.render(scenes[si], sensor=sen, outputs=OUTS[kind], **opts)
            torch.cuda.synchronize()
            done.append((kind, arr, time.monotonic() - t0, frame_rays(kind, sen)))
        return done

    def served_run(arrivals, srv):
        frames = [(arrivals[k], f) for k, tk in enumerate(ticks) for f in tk]
        t0 = time.monotonic()
        pending, done = {}, []
        i = 0
        while len(done) < len(frames):
            now = time.monotonic() - t0
            while i < len(frames) and frames[i][0] <= now:
                arr, (kind, sen, si) = frames[i]
                pending[srv.submit(scenes[si], sen, outputs=OUTS[kind], **opts)] = (kind, arr, frame_rays(kind, sen))
                i += 1
            # requests complete about in submission order (FIFO admission, launches in order):
            # poll the oldest ones
            for tk in list(itertools.islice(pending, 64)):
                r = srv.poll(tk)
                if r is None:
                    continue
                kind, arr, n = pending.pop(tk)
                done.append((kind, arr, r[2] - t0, n))
                srv.release(tk)
            if pending or i < len(frames):
                time.sleep(0.0002)
        return done

    def summarize(done, warm_frames):
        done = sorted(done, key=lambda d: d[1])[warm_frames:]
        lat = np.array([d[2] - d[1] for d in done]) * 1e3
        span = max(d[2] for d in done) - min(d[1] for d in done)
        rays = sum(d[3] for d in done)
        per = {}
        for kind in ("camera", "fisheye", "lidar"):
            l = np.array([d[2] - d[1] for d in done if d[0] == kind]) * 1e3
            per[kind] = {"p50_ms": round(float(np.percentile(l, 50)), 2), "p99_ms": round(float(np.percentile(l, 99)), 2)}
        return {"mrays_s": round(rays / span / 1e6, 1), "p50_ms": round(float(np.percentile(lat, 50)), 2),
                "p99_ms": round(float(np.percentile(lat, 99)), 2), "by_sensor": per}

    warm_frames = warm_ticks * 10
    # plain capacity: closed loop (every tick queued at t = 0)
    closed = [0.0] * len(ticks)
    progress("serving: plain, closed loop")
    plain_closed = summarize(plain_run(closed), warm_frames)
    rays_per_tick = sum(frame_rays(k, s) for k, s, _ in ticks[0])
    lam_p = plain_closed["mrays_s"] * 1e6 / rays_per_tick      # ticks per second the plain path sustains
    pool = int(pool_gib * (1 << 30))
    servers = {name: salf.Server(pool_bytes=pool, device=dev, max_batch=mb, max_inflight=mi, max_launch_rays=mr)
               for name, (mb, mi, mr) in configs.items()}
    closed_loop = {"plain": plain_closed}
    for name, srv in servers.items():
        progress(f"serving: {name}, closed loop")
        closed_loop[name] = summarize(served_run(closed, srv), warm_frames)
    points = []
    for load in (0.5, 0.9, 1.5):
        gaps = rng.exponential(1.0 / (load * lam_p), size=len(ticks))
        arrivals = list(np.cumsum(gaps) - gaps[0])
        progress(f"serving: Poisson arrivals at {load} x the plain capacity")
        pt = {"load": load, "ticks_per_s": round(load * lam_p, 2), "plain": summarize(plain_run(arrivals), warm_frames)}
        for name, srv in servers.items():
            pt[name] = summarize(served_run(arrivals, srv), warm_frames)
        points.append(pt)
    stats = {}
    for name, srv in servers.items():
        st = srv.stats()
        stats[name] = {"max_batch": configs[name][0], "max_inflight": configs[name][1],
                       "max_launch_rays": configs[name][2], "launches": st["launches"], "pool_peak": st["pool_peak"]}
        srv.close()
    return {"workload": "4 resident driving scenes (seeds 11-14); Poisson vehicle ticks of 6 pinhole 1920x1080 + "
                        "2 fisheye 1280x960 (190 deg) with 30 us/row rolling shutter + 2 LiDAR 64x2048",
            "rays_per_tick": rays_per_tick, "ticks": n_ticks, "warmup_ticks": warm_ticks,
            "pool_bytes": pool, "plain_capacity_ticks_per_s": round(lam_p, 2),
            "closed_loop": closed_loop, "poisson": points, "servers": stats}


# ------------------------------------------------------------------ training step (differentiation)
# hits stored per ray by the training forward (camera and LiDAR batches), whose backward then reads
# them instead of walking the scene again; a ray with more hits is walked
HIT_CAPACITY = 256


def training_bench(salf, torch, dev, data, steps=10, seed=4):
    """1,048,576 rays per batch on the driving scene: 80% camera pixels drawn from 8 random views,
    20% LiDAR rays from 2 sweeps; loss = mean squared colour error + mean absolute depth error
    against targets rendered from a perturbed copy (logits + N(0, 0.1^2)).  A step = zero the
    gradients, forward, loss gradients, hand-written backward, an SGD update of every corner logit
    and the refresh of the activated corner values the renders read.  The timed step runs the
    LiDAR batch's forward and backward on a second stream beside the camera batch's (the two
    backwards add into the same gradient with atomics); the same step on one stream gives the
    forward / backward split."""
    import numpy as np

    import synth
    rng = np.random.default_rng(seed)
    scene = salf.Scene.from_data(data, device=dev, preactivate=True)
    pert = synth.SceneData(**{**data.__dict__})
    prng = np.random.default_rng(5)
    pert.z_geo = (data.z_geo + prng.normal(0, 0.1, data.z_geo.shape)).astype(np.float32)
    pert.z_rgb = (data.z_rgb + prng.normal(0, 0.1, data.z_rgb.shape)).astype(np.float32)
    pert.z_int = (data.z_int + prng.normal(0, 0.1, data.z_int.shape)).astype(np.float32)
    target_scene = salf.Scene.from_data(pert, device=dev)
    n_cam, n_lid = 838861, 209715
    oc, dc = [], []
    for _ in range(8):
        x, y = rng.uniform(-80, 80), rng.uniform(-3, 3)
        yaw = rng.uniform(-30, 30) + (0.0 if rng.random() < 0.5 else 180.0)
        r = salf.generate_rays(synth.pinhole(1920, 1080, 60.0, synth.yaw_pitch_camera(yaw, -5.0), (x, y, 1.6)), dev)
        oc.append(r["o"])
        dc.append(r["d"])
    oc, dc = torch.cat(oc), torch.cat(dc)
    # the sampled pixels are batched in 16x16 screen blocks (ray bundles; at 5% of the pixels a wave's
    # 64 rays cover about one block), so that the rays of one wave see neighbouring voxels as in a
    # frame render (8x8 blocks: forward and backward ~2-4% slower)
    ic = np.sort(rng.choice(oc.shape[0], n_cam, replace=False))
    view, pix = ic // (1920 * 1080), ic % (1920 * 1080)
    py, px = pix // 1920, pix % 1920
    ic = ic[np.lexsort((px % 16, py % 16, px // 16, py // 16, view))]
    ic = torch.from_numpy(ic).to(dev)
    ol, dl = [], []
    for x in (-60.0, 20.0):
        r = salf.generate_rays(synth.lidar_spinning(64, 2048, -25, 15, np.eye(3), (x, 0.37, 1.85), 0.1, v=(10, 0, 0)),
                               dev)
        ol.append(r["o"])
        dl.append(r["d"])
    ol, dl = torch.cat(ol), torch.cat(dl)
    il = np.sort(rng.choice(ol.shape[0], n_lid, replace=False))
    sweep, pix = il // (64 * 2048), il % (64 * 2048)
    beam, col = pix // 2048, pix % 2048
    il = il[np.lexsort((col % 32, beam % 2, col // 32, beam // 2, sweep))]  # 32 columns x 2 beams
    il = torch.from_numpy(il).to(dev)
    oc, dc = oc[ic].contiguous(), dc[ic].contiguous()
    ol, dl = ol[il].contiguous(), dl[il].contiguous()
    opts = dict(samples=4, t_min=1e-6)
    tgt_c = salf.render(target_scene, o=oc, d=dc, outputs=("rgb",), **opts)["rgb"]
    tgt_d = salf.render(target_scene, o=ol, d=dl, outputs=("depth",), **opts)["depth"]
    d_geo, d_rgb, d_int = (torch.zeros_like(t) for t in (scene.geo, scene.rgb, scene.intensity))
    saved_outs = ("rgb", "depth", "opacity", "t_end", "n_hits")
    lr = 100.0

    def step(ev=None, cap=HIT_CAPACITY):
        d_geo.zero_()
        d_rgb.zero_()
        # the forwards store each ray's hits, which the backwards read instead of walking again
        fc = salf.render(scene, o=oc, d=dc, outputs=saved_outs, hit_capacity=cap, **opts)
        fl = salf.render(scene, o=ol, d=dl, outputs=("depth", "opacity", "t_end", "n_hits"), hit_capacity=cap, **opts)
        g_c = (2.0 / (3 * n_cam)) * (fc["rgb"] - tgt_c)
        g_l = (1.0 / n_lid) * torch.sign(fl["depth"] - tgt_d)
        if ev is not None:
            ev.record()
        salf.render_backward(scene, fc, {"rgb": g_c}, o=oc, d=dc, d_geo=d_geo, d_rgb=d_rgb, **opts)
        salf.render_backward(scene, fl, {"depth": g_l}, o=ol, d=dl, d_geo=d_geo, **opts)
        scene.geo.add_(d_geo, alpha=-lr)
        scene.rgb.add_(d_rgb, alpha=-lr)
        scene.refresh()
        return fc, fl

    side = torch.cuda.Stream(device=dev)  # default priority

    def step_two_streams(cap=HIT_CAPACITY):
        main = torch.cuda.current_stream(dev)
        d_geo.zero_()
        d_rgb.zero_()
        side.wait_stream(main)  # the previous update and the cleared gradients
        with torch.cuda.stream(side):
            fl = salf.render(scene, o=ol, d=dl, outputs=("depth", "opacity", "t_end", "n_hits"), hit_capacity=cap,
                             **opts)
            g_l = (1.0 / n_lid) * torch.sign(fl["depth"] - tgt_d)
            salf.render_backward(scene, fl, {"depth": g_l}, o=ol, d=dl, d_geo=d_geo, **opts)
        fc = salf.render(scene, o=oc, d=dc, outputs=saved_outs, hit_capacity=cap, **opts)
        g_c = (2.0 / (3 * n_cam)) * (fc["rgb"] - tgt_c)
        salf.render_backward(scene, fc, {"rgb": g_c}, o=oc, d=dc, d_geo=d_geo, d_rgb=d_rgb, **opts)
        main.wait_stream(side)
        scene.geo.add_(d_geo, alpha=-lr)
        scene.rgb.add_(d_rgb, alpha=-lr)
        scene.refresh()
        return fc, fl

    for _ in range(2):
        step()
        step_two_streams()
    torch.cuda.synchronize()
    times, fwd = [], []
    for _ in range(steps):
        e0, em, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        fc, fl = step(em)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        fwd.append(e0.elapsed_time(em))
    grad_abs_sum = float(d_geo.abs().sum() + d_rgb.abs().sum())
    times2 = []
    for _ in range(steps):
        e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
        e0.record()
        fc, fl = step_two_streams()
        e1.record()
        torch.cuda.synchronize()
        times2.append(e0.elapsed_time(e1))
    loss = float(torch.mean((fc["rgb"] - tgt_c) ** 2) + torch.mean(torch.abs(fl["depth"] - tgt_d)))
    ms_serial = float(np.median(times))
    ms = float(np.median(times2))
    # the same step with both backwards walking the scene again (no stored hits), for comparison
    walk_times, walk_fwd = [], []
    for _ in range(steps // 2 + 1):
        e0, em, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        step(em, cap=0)
        e1.record()
        torch.cuda.synchronize()
        walk_times.append(e0.elapsed_time(e1))
        walk_fwd.append(e0.elapsed_time(em))
    refine = refine_pass(salf, torch, scene, d_rgb, data)
    g_c = (2.0 / (3 * n_cam)) * (fc["rgb"] - tgt_c)
    g_l = (1.0 / n_lid) * torch.sign(fl["depth"] - tgt_d)
    paper = paper_field_pass(salf, torch, dev, data, oc, dc, ol, dl, g_c, g_l, opts, steps)
    sdf = paper_field_pass(salf, torch, dev, data, oc, dc, ol, dl, g_c, g_l, opts, steps, field="sdf")
    return {"workload": "driving scene, 838,861 camera pixels (8 random views) + 209,715 LiDAR rays (2 sweeps), "
                        "batched in 16x16 pixel blocks / 32x2 LiDAR tiles, L2 colour + L1 depth vs a perturbed copy, "
                        "SGD update + activation refresh in the step; the forwards store each ray's hits "
                        f"(up to {HIT_CAPACITY}) and the backwards read them; the LiDAR batch on a second stream",
            "rays": n_cam + n_lid, "ms_per_step_median": round(ms, 3),
            "one_stream": {"ms_per_step_median": round(ms_serial, 3),
                           "forward_ms_median": round(float(np.median(fwd)), 3),
                           "backward_ms_median": round(ms_serial - float(np.median(fwd)), 3)},
            "walking_backward": {"ms_per_step_median": round(float(np.median(walk_times)), 3),
                                 "forward_ms_median": round(float(np.median(walk_fwd)), 3),
                                 "backward_ms_median": round(float(np.median(walk_times)) - float(np.median(walk_fwd)), 3)},
            "mrays_s_fwd_bwd": round((n_cam + n_lid) / ms / 1e3, 2), "loss": round(loss, 5),
            "grad_abs_sum": grad_abs_sum, "paper_field": paper, "sdf_field": sdf, "refine": refine}


def refine_pass(salf, torch, scene, d_rgb, data):
    """Densification and pruning after a training step (Sec. 3.3): split the 5% of touched voxels
    with the largest colour gradient (L1), prune alpha < 0.001, then build the refined scene (with
    its dense leaf index).  Wall-clock times; both calls block."""
    import time

    import numpy as np
    l1 = d_rgb.abs().sum((1, 2))
    touched = l1[l1 > 0]
    thr = float(torch.quantile(touched[:1 << 24].float(), 0.95)) if touched.numel() else 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = scene.refine(d_rgb, thr, 1e-3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    new = salf.Scene(out["voxels"], out["geo"], out["rgb"], out["intensity"], data.origin, data.root_size,
                     data.root_dims, data.max_level, preactivate=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    n_in, n_out = scene.n, new.n
    n_split = int((l1 > thr).sum())
    new.destroy()
    return {"voxels_in": n_in, "voxels_out": n_out, "split_threshold_l1": thr, "refine_ms": round((t1 - t0) * 1e3, 3),
            "rebuild_ms": round((t2 - t1) * 1e3, 3),
            "note": f"{n_split} voxels over the threshold (those at the finest level stay whole)"}


def actors_pass(salf, torch, dev, data, scene, cam, opts, steps, n_actors=7):
    """The camera frame with dynamic actors (Sec. 4.1): n_actors car-sized scenes (4.8 x 2.4 x 2.4 m,
    seeded, voxels to 0.15 m) on the road ahead of the camera, each yawed by a seeded angle and
    placed where its box holds no background voxel, rendered with salf_render_composite beside the
    plain frame.  HIP-event times per frame."""
    import numpy as np

    import synth
    rng = np.random.default_rng(8)
    lo_f, hi_f = data.finest_bounds()
    gs = (1 << data.max_level) / data.root_size
    vlo = data.origin + lo_f / gs                       # world bounds of every background voxel
    vhi = data.origin + hi_f / gs
    ext = np.array([4.8, 2.4, 2.4])
    actors, poses = [], []
    x = -86.0
    while len(actors) < n_actors and x < 0.0:
        yaw = np.radians(rng.uniform(-15.0, 15.0))
        c, s_ = np.cos(yaw), np.sin(yaw)
        R = np.array([[c, -s_, 0.0], [s_, c, 0.0], [0.0, 0.0, 1.0]])
        centre = np.array([x, 1.75 if len(actors) % 2 else -1.75, 0.35 + ext[2] / 2])
        half = np.abs(R) @ (ext / 2) + 0.05             # world half-extent of the rotated box, with margin
        if not np.any(np.all((vlo < centre + half) & (vhi > centre - half), axis=1)):
            a = synth.random_scene(300 + len(actors), root_dims=(4, 2, 2), max_level=3, root_size=1.2,
                                   origin=(0.0, 0.0, 0.0), fill=0.7)
            t = (centre - R @ (ext / 2)).astype(np.float32)
            actors.append(salf.Scene.from_data(a, device=dev, preactivate=True))
            poses.append((R.astype(np.float32), t))
        x += 6.0
    items = [(sc, R, t) for sc, (R, t) in zip(actors, poses)]
    outs = ("rgb", "depth", "opacity")

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    plain = timed(lambda: salf.render(scene, sensor=cam, outputs=outs, **opts))
    comp = timed(lambda: salf.render_composite(scene, items, sensor=cam, outputs=outs, **opts))
    hits = salf.render_composite(scene, items, sensor=cam, outputs=("n_hits",), **opts)["n_hits"]
    base = salf.render(scene, sensor=cam, outputs=("n_hits",), **opts)["n_hits"]
    rec = {"n_actors": len(actors), "actor_voxels": int(sum(a.n for a in actors)),
           "camera_ms_plain": round(plain, 4), "camera_ms_with_actors": round(comp, 4),
           "pixels_changed_by_actors": int((hits != base).sum())}
    for a in actors:
        a.destroy()
    return rec


def batched_pass(salf, torch, dev, scene, cam, lid, steps):
    """The step's camera frame and LiDAR sweep submitted to the server each tick, so that both
    sensors' tiles go out in one cost-ordered batched launch, two ticks in flight (the server's
    host round trip between launches hidden).  Wall time per tick over `steps` ticks, after 3."""
    import time as _t
    srv = salf.Server(1 << 30, device=dev, max_batch=2, max_inflight=2)
    n = cam["width"] * cam["height"] + lid["width"] * lid["height"]

    def tick():
        return (srv.submit(scene, cam, outputs=("rgb", "depth", "opacity")),
                srv.submit(scene, lid, outputs=("depth", "intensity", "opacity")))

    def drain(ts):
        for a, b in ts:
            srv.wait(a)
            srv.wait(b)
            srv.release(a)
            srv.release(b)

    drain([tick() for _ in range(3)])
    torch.cuda.synchronize()
    launches0 = srv.stats()["launches"]
    t0 = _t.perf_counter()
    drain([tick() for _ in range(steps)])
    torch.cuda.synchronize()
    dt = (_t.perf_counter() - t0) / steps
    launches = srv.stats()["launches"] - launches0
    srv.close()
    return {"ms_per_tick": round(dt * 1e3, 4), "mrays_s": round(n / dt / 1e6, 1), "ticks": steps,
            "launches": launches}


def raster_pass(salf, torch, dev, scene, steps, opts):
    """Tile-based splatting (Sec. 3.2) against ray casting of the same global-shutter pinhole on the
    driving scene, across resolutions (the paper's ray-vs-raster trade-off, Sec. 5.2): per frame,
    wall time of the splatting call (projection, scan, the pair-count read-back, sort, tiles; it
    blocks once) and of the ray cast with its schedule, both to a synchronized stream, after 2
    warm-up frames.  Outputs are the same bits (checked here on the full-HD frame)."""
    import time as _t

    import synth
    rec = []
    outs = ("rgb", "depth", "opacity")
    for w, h in ((480, 270), (960, 540), (1920, 1080), (3840, 2160)):
        cam = synth.config1_camera(w, h)
        n = w * h
        out_r = {"rgb": torch.empty((n, 3), device=dev), "depth": torch.empty(n, device=dev),
                 "opacity": torch.empty(n, device=dev)}
        out_c = {k: torch.empty_like(v) for k, v in out_r.items()}

        def ray():
            salf.render(scene, sensor=cam, outputs=outs, out=out_c, **opts)

        def splat():
            salf.render_raster(scene, cam, outputs=outs, out=out_r, **opts)

        res = {"width": w, "height": h}
        for name, fn in (("ray", ray), ("raster", splat)):
            for _ in range(2):
                fn()
            torch.cuda.synchronize()
            t0 = _t.perf_counter()
            for _ in range(steps):
                fn()
            torch.cuda.synchronize()
            res[f"{name}_ms"] = round((_t.perf_counter() - t0) / steps * 1e3, 4)
        res["pairs"] = int(scene.raster_pairs)
        if w == 1920:
            res["same_bits"] = bool(all(torch.equal(out_r[k], out_c[k]) for k in outs))
        rec.append(res)
    return {"workload": "driving scene (pre-activated), pinhole from the driving camera pose, S=4, t_min=1e-6",
            "frames": rec}


def paper_field_pass(salf, torch, dev, data, oc, dc, ol, dl, g_c, g_l, opts, steps, seed=6, field="paper"):
    """Forward and backward of the same batch on the driving scene's voxels with the paper's field
    (Eq. 1-2): seeded parameters, density slopes N(0, 0.5^2) and offset N(0, 1) - 1, colour and
    intensity slopes and SH coefficients N(0, 0.5^2), offsets N(0, 1).  field="sdf": the density
    of Eq. 5-6 instead, signed-distance slopes N(0, 0.6^2) and offset N(0, 0.5^2), log a ~
    N(0.5, 0.3^2), log b ~ N(-1, 0.3^2).  Timed by HIP events; no update."""
    import numpy as np

    import synth
    rng = np.random.default_rng(seed)
    n = data.n
    geo = np.zeros((n, 8), np.float32)
    geo[:, :3] = rng.normal(0, 0.5, (n, 3))
    geo[:, 3] = rng.normal(0, 1, n) - 1.0
    if field == "sdf":
        geo[:, :3] = rng.normal(0, 0.6, (n, 3))
        geo[:, 3] = rng.normal(0, 0.5, n)
        geo[:, 4] = rng.normal(0.5, 0.3, n)
        geo[:, 5] = rng.normal(-1.0, 0.3, n)
    rgb = np.zeros((n, 3, 8), np.float32)
    rgb[:, :, :3] = rng.normal(0, 0.5, (n, 3, 3))
    rgb[:, :, 3] = rng.normal(0, 1, (n, 3))
    rgb[:, :, 4:7] = rng.normal(0, 0.5, (n, 3, 3))
    ity = np.zeros((n, 8), np.float32)
    ity[:, :3] = rng.normal(0, 0.5, (n, 3))
    ity[:, 3] = rng.normal(0, 1, n)
    pdata = synth.SceneData(**{**data.__dict__, "z_geo": geo, "z_rgb": rgb, "z_int": ity})
    scene = salf.Scene.from_data(pdata, device=dev, field=field)
    d_geo, d_rgb = torch.zeros_like(scene.geo), torch.zeros_like(scene.rgb)
    outs = ("rgb", "depth", "opacity", "t_end", "n_hits")
    fwd, bwd = [], []
    for i in range(steps + 2):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        fc = salf.render(scene, o=oc, d=dc, outputs=outs, hit_capacity=HIT_CAPACITY, **opts)
        fl = salf.render(scene, o=ol, d=dl, outputs=("depth", "opacity", "t_end", "n_hits"), hit_capacity=HIT_CAPACITY,
                         **opts)
        e1.record()
        salf.render_backward(scene, fc, {"rgb": g_c}, o=oc, d=dc, d_geo=d_geo, d_rgb=d_rgb, **opts)
        salf.render_backward(scene, fl, {"depth": g_l}, o=ol, d=dl, d_geo=d_geo, **opts)
        e2.record()
        torch.cuda.synchronize()
        if i >= 2:
            fwd.append(e0.elapsed_time(e1))
            bwd.append(e1.elapsed_time(e2))
    scene.destroy()
    return {"forward_ms_median": round(float(np.median(fwd)), 3), "backward_ms_median": round(float(np.median(bwd)), 3),
            "shaded_hits_per_camera_ray": round(float(fc["n_hits"].double().mean()), 3)}


def touched_voxels(salf, torch, scene, sensor, opts):
    """Distinct voxels a render of `sensor` shades (the compulsory parameter reads): the voxels
    whose density gradient is non-zero in the backward of an opacity loss, where every shaded voxel
    receives T_end x its segment length x positive corner weights."""
    outs = ("opacity", "t_end", "n_hits")
    fwd = salf.render(scene, sensor=sensor, outputs=outs, **opts)
    g = {"opacity": torch.ones_like(fwd["opacity"])}
    d_geo, _, _ = salf.render_backward(scene, fwd, g, sensor=sensor, **opts)
    n = int((d_geo != 0).any(dim=1).sum())
    del d_geo
    return n


def copy_bandwidth(torch, dev, nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (bytes read + written per second, GB/s) of a 1 GiB buffer."""
    src = torch.ones(nbytes // 4, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


# ------------------------------------------------------------------ HBM counter pass
COPY_BYTES = 512 << 20


def counter_pass(salf, torch, dev, data, what="multi"):
    """Kernels for a rocprofv3 --pmc run: a plain device copy of COPY_BYTES (reads and writes
    exactly that many bytes: the counters' calibration), then three launches of `what` on the
    pre-activated driving scene: "camera" the frame's render (the roofline's kernel), "lidar" the
    sweep's, "multi" both in one launch, "backward" the camera frame's backward (corner field,
    colour gradient) reading the hits its forward stored, as the training step does,
    "backward_walk" the same backward walking the scene again."""
    import synth
    src = torch.ones(COPY_BYTES // 4, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    scene = salf.Scene.from_data(data, device=dev, preactivate=True)
    cam, lid = synth.config1_camera(), synth.config2_lidar()
    n_cam, n_lid = cam["width"] * cam["height"], lid["width"] * lid["height"]
    cam_out = {"rgb": torch.empty((n_cam, 3), device=dev), "depth": torch.empty(n_cam, device=dev),
               "opacity": torch.empty(n_cam, device=dev)}
    lid_out = {k: torch.empty(n_lid, device=dev) for k in ("depth", "intensity", "opacity")}
    opts = dict(samples=4, t_min=1e-6)
    saved = None
    if what.startswith("backward"):
        saved = salf.render(scene, sensor=cam, outputs=("rgb", "depth", "opacity", "t_end", "n_hits"),
                            hit_capacity=HIT_CAPACITY if what == "backward" else 0, **opts)
        grads = {"rgb": torch.full_like(saved["rgb"], 1e-3)}
        d_geo, d_rgb = torch.zeros_like(scene.geo), torch.zeros_like(scene.rgb)
    for _ in range(3):
        if what == "multi":
            salf.render_multi([(scene, cam, cam_out), (scene, lid, lid_out)], **opts)
        elif what == "camera":
            salf.render(scene, sensor=cam, outputs=cam_out.keys(), out=cam_out, **opts)
        elif what == "lidar":
            salf.render(scene, sensor=lid, outputs=lid_out.keys(), out=lid_out, **opts)
        else:
            salf.render_backward(scene, saved, dict(grads), sensor=cam, d_geo=d_geo, d_rgb=d_rgb, **opts)
    torch.cuda.synchronize()
    rays = {"multi": n_cam + n_lid, "camera": n_cam, "lidar": n_lid, "backward": n_cam, "backward_walk": n_cam}[what]
    print(json.dumps({"counter_pass": what, "copy_bytes": COPY_BYTES, "rays": rays,
                      "kernel_source_hash": kernel_source_hash()}), flush=True)


def progress(msg):
    """One line on stderr per stage of the run (the JSON record alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


# ------------------------------------------------------------------ GPU
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-training", action="store_true")
    ap.add_argument("--serve-ticks", type=int, default=500)
    ap.add_argument("--counter-pass", choices=("multi", "camera", "lidar", "backward", "backward_walk"), default=None,
                    help="run only the kernels a rocprofv3 --pmc pass needs: a 512 MiB device copy (the "
                         "calibration of the HBM byte counters) and 3 launches of the named render")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the path runs on a single "
              f"GPU; sharding across GPUs is not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2507_18713_amd as salf
    import synth

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    data = synth.config1_scene()
    t_gen = time.perf_counter() - t0
    if args.counter_pass:
        counter_pass(salf, torch, dev, data, args.counter_pass)
        return
    # forward renders read the activated corner values stored at upload (the workload's corner
    # values are softplus / sigmoid of the drawn logits); the raw-logit scene is timed beside it
    scene = salf.Scene.from_data(data, device=dev, preactivate=True)
    raw_scene = salf.Scene.from_data(data, device=dev)
    torch.cuda.synchronize()
    # scene build time alone (upload excluded)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    scene2 = salf.Scene(scene._voxels, scene.geo, scene.rgb, scene.intensity, data.origin, data.root_size,
                        data.root_dims, data.max_level, preactivate=True)
    e1.record()
    torch.cuda.synchronize()
    build_ms = e0.elapsed_time(e1)
    scene2.destroy()
    del scene2

    cam = synth.config1_camera()
    lid = synth.config2_lidar()
    n_cam, n_lid = cam["width"] * cam["height"], lid["width"] * lid["height"]
    opts = dict(samples=4, t_min=1e-6)
    cam_out = {"rgb": torch.empty((n_cam, 3), device=dev), "depth": torch.empty(n_cam, device=dev),
               "opacity": torch.empty(n_cam, device=dev)}
    lid_out = {k: torch.empty(n_lid, device=dev) for k in ("depth", "intensity", "opacity")}

    main_stream = torch.cuda.current_stream(dev)
    side_stream = torch.cuda.Stream(device=dev)  # default priority

    def step(ev=None):
        # the LiDAR sweep of a step runs on a second stream beside its camera frame; a step
        # starts once the previous step's two renders have finished.  Every step builds the camera
        # frame's tile schedule (a frame's pose may change) and renders with it.  ev: events
        # around the schedule and the camera render (main stream) and the LiDAR render (second
        # stream)
        side_stream.wait_stream(main_stream)
        if ev is not None:
            ev[0].record(main_stream)
        sched = salf.render_schedule(scene, sensor=cam)
        if ev is not None:
            ev[1].record(main_stream)
        salf.render(scene, sensor=cam, outputs=cam_out.keys(), out=cam_out, schedule=sched, **opts)
        if ev is not None:
            ev[2].record(main_stream)
        with torch.cuda.stream(side_stream):
            if ev is not None:
                ev[3].record(side_stream)
            salf.render(scene, sensor=lid, outputs=lid_out.keys(), out=lid_out, **opts)
            if ev is not None:
                ev[4].record(side_stream)
        main_stream.wait_stream(side_stream)

    def kernel_ms(sensor, outs, pieces=1):
        """Average duration of one render alone (its schedule built beforehand), by HIP events on
        the stream it runs on."""
        sched = salf.render_schedule(scene, sensor=sensor)
        salf.render(scene, sensor=sensor, outputs=outs.keys(), out=outs, schedule=sched, pieces=pieces, **opts)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(args.steps):
            salf.render(scene, sensor=sensor, outputs=outs.keys(), out=outs, schedule=sched, pieces=pieces, **opts)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / args.steps

    # instrumented run (not timed): shaded hits per ray for the algorithmic byte count
    hc = salf.render(scene, sensor=cam, outputs=("n_hits",), **opts)["n_hits"]
    hl = salf.render(scene, sensor=lid, outputs=("n_hits",), **opts)["n_hits"]
    hits_cam, hits_lid = int(hc.sum().item()), int(hl.sum().item())

    items = [(scene, cam, cam_out), (scene, lid, lid_out)]

    def multi_step(ev=None):
        # the camera frame and the LiDAR sweep in one launch (salf_render_multi): both sensors'
        # tiles, heaviest first, pulled by one grid; ev: events around the call (its batch schedule
        # and the render kernel) on the stream it runs on
        if ev is not None:
            ev[0].record(main_stream)
        salf.render_multi(items, **opts)
        if ev is not None:
            ev[1].record(main_stream)

    progress("timed steps (two streams)")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    # per-launch durations inside the timed region (each render shares the GPU with the other)
    sched_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    cam_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps
    lid_ms = sum(e[3].elapsed_time(e[4]) for e in evs) / args.steps
    # steady-state period: camera start to camera start (steps are serialized by the stream waits)
    step_ms = evs[0][0].elapsed_time(evs[-1][0]) / (args.steps - 1) if args.steps > 1 else None

    progress("timed steps (one launch per step)")
    for _ in range(args.warmup):
        multi_step()
    torch.cuda.synchronize()
    mevs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    t_start = time.perf_counter()
    for i in range(args.steps):
        multi_step(mevs[i])
    torch.cuda.synchronize()
    wall_multi = time.perf_counter() - t_start
    multi_ms = sum(e[0].elapsed_time(e[1]) for e in mevs) / args.steps
    rays = n_cam + n_lid
    value = rays / (wall / args.steps) / 1e6
    value_multi = rays / (wall_multi / args.steps) / 1e6
    # each render alone, after the timed region
    cam_alone_ms = kernel_ms(cam, cam_out)
    lid_alone_ms = kernel_ms(lid, lid_out)
    # the sweep alone with each ray's root cells shared out among P lanes (opts.pieces)
    lid_pieces_ms = {P: kernel_ms(lid, lid_out, pieces=P) for P in (2, 4, 8)}

    # the same camera frame from the raw-logit scene (corner activations evaluated per hit)
    e0.record()
    for _ in range(args.steps):
        salf.render(raw_scene, sensor=cam, outputs=cam_out.keys(), out=cam_out, **opts)
    e1.record()
    torch.cuda.synchronize()
    cam_raw_ms = e0.elapsed_time(e1) / args.steps
    progress("actors")
    actors_rec = actors_pass(salf, torch, dev, data, scene, cam, opts, args.steps)
    progress("splatting vs ray casting")
    raster_rec = raster_pass(salf, torch, dev, scene, max(3, args.steps // 2), opts)
    progress("batched step")
    batched_rec = None if args.no_serving else batched_pass(salf, torch, dev, scene, cam, lid, args.steps)

    cam_bytes = hits_cam * CAM_HIT_BYTES + n_cam * CAM_RAY_BYTES
    lid_bytes = hits_lid * LID_HIT_BYTES + n_lid * LID_RAY_BYTES
    achieved = cam_bytes / (cam_ms * 1e-3) / 1e9
    multi_achieved = (cam_bytes + lid_bytes) / (multi_ms * 1e-3) / 1e9
    traffic = measured_traffic(n_cam, CAMERA_TRAFFIC_FILE)
    multi_traffic = measured_traffic(n_cam + n_lid)
    progress("compulsory bytes and copy bandwidth")
    unique_cam = touched_voxels(salf, torch, scene, cam, opts)
    unique_lid = touched_voxels(salf, torch, scene, lid, opts)
    copy_gbs = copy_bandwidth(torch, dev)
    rec = {
        "metric": "Mrays/s camera+LiDAR render on 1 GPU",
        "value": round(value, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "driving scene (2.01M voxels, 5 levels 1.6-0.1 m) + 1920x1080 pinhole frame + "
                        "64x2048 rolling-shutter LiDAR sweep, S=4, t_min=1e-6",
            "n_voxels": int(data.n), "camera_rays": n_cam, "lidar_rays": n_lid, "samples_per_voxel": 4,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "render_kernel, camera frame (launched on the main stream; the LiDAR sweep's render "
                      "runs beside it on a second stream)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "launch_ms": round(cam_ms, 4),
            "algorithmic_bytes": cam_bytes,
            "compulsory_bytes": unique_cam * CAM_HIT_BYTES + n_cam * CAM_RAY_BYTES,
            "unique_voxels_shaded": {"camera": unique_cam, "lidar": unique_lid},
            "copy_GBs": round(copy_gbs, 1),
            "frac_of_copy": round(achieved / copy_gbs, 4),
        },
        "one_launch_step": {
            "value": round(value_multi, 3), "ms_per_step": round(wall_multi / args.steps * 1e3, 4),
            "launch_ms": round(multi_ms, 4),
            "achieved_GBs": round(multi_achieved, 1), "frac": round(multi_achieved / HBM_PEAK_GBS, 4),
            "traffic": multi_traffic,
            "note": "camera frame and LiDAR sweep tiles in one render_batch_kernel launch (salf_render_multi); "
                    "the event window also holds its batch schedule's two small kernels",
        },
        "camera": {"ms": round(cam_ms, 4), "mrays_s": round(n_cam / cam_ms / 1e3, 2),
                   "ms_alone": None if cam_alone_ms is None else round(cam_alone_ms, 4),
                   "schedule_ms": round(sched_ms, 4),
                   "ms_raw_logit_scene": round(cam_raw_ms, 4),
                   "shaded_hits_per_ray": round(hits_cam / n_cam, 3), "algorithmic_bytes": cam_bytes},
        "lidar": {"ms": round(lid_ms, 4), "mrays_s": round(n_lid / lid_ms / 1e3, 2),
                  "ms_alone": None if lid_alone_ms is None else round(lid_alone_ms, 4),
                  "shaded_hits_per_ray": round(hits_lid / n_lid, 3), "algorithmic_bytes": lid_bytes,
                  "achieved_GBs": round(lid_bytes / (lid_ms * 1e-3) / 1e9, 1),
                  "sweeps_per_s_alone": None if lid_alone_ms is None else round(1e3 / lid_alone_ms, 1),
                  "ms_alone_in_pieces": {str(P): round(v, 4) for P, v in lid_pieces_ms.items()},
                  "sweeps_per_s_alone_in_pieces": {str(P): round(1e3 / v, 1) for P, v in lid_pieces_ms.items()}},
        "event_ms_per_step": None if step_ms is None else round(step_ms, 4),
        "step": "camera render (its tile schedule built in the step) and LiDAR render on two streams",
        "scene_build_ms": round(build_ms, 3),
        "actors": actors_rec,
        "raster_vs_ray": raster_rec,
        "batched_step": batched_rec,
        "dense_index_bytes": int(scene.index.numel()) if scene.index is not None else 0,
        "scene_generate_s": round(t_gen, 2),
        "kernel_source_hash": kernel_source_hash(),
    }
    if not args.no_training:
        progress("training step")
        rec["training"] = training_bench(salf, torch, dev, data)
    if not args.no_serving:
        progress("serving")
        rec["serving"] = serving_bench(salf, torch, dev, n_ticks=args.serve_ticks)
        rec["metric"] = "Mrays/s camera+LiDAR render on 1 GPU; p50/p99 frame latency served vs plain"
    if not args.no_cpu_baseline:
        progress("cpu baseline")
        rec["cpu_baseline"] = cpu_baseline()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
