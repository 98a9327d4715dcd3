"""Benchmark: frames/s and p50/p99 frame latency of the forward 3DGS rasterizer.

Workload: 3M Gaussians (64 anisotropic clusters + 40% flattened surface
splats, SH degree 3), 1920x1080, the 300-pose smooth 6DoF trajectory, with
the attributes stored in FP32 (the headline value) and in FP16 / BF16.
A step is one frame: preprocess, scan, duplicate, radix sort, tile ranges,
blend + RGB8 pack, with the scene resident in HBM and the frame written to a
device buffer.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 300] [--warmup 10] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import math
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (packed FMA), TFLOP/s
# FP32 flops of one (pixel, Gaussian) evaluation in the blend: offsets (2),
# exponent polynomial (3 mul/fma = 8 flops incl. 2 plain mul), exp2 (1), clamp
# (1); a contribution adds transmittance (2), weight (1), 3 FMA colour (6)
FLOPS_EVAL = 12
FLOPS_CONTRIB = 9
# the cost model of the scope table: 15 VALU operations + 1 exp per evaluation
OPS_EVAL_MODEL = 16


def _stats(ts):
    a = np.asarray(ts) * 1e3
    return float(np.median(a)), float(np.percentile(a, 99))


def pose_index(i, steps, n_poses):
    """Timed frame i of `steps` renders pose pose_index(...) of the trajectory:
    fewer steps than poses are spread evenly over the whole trajectory (every
    n_poses/steps-th pose), more wrap around it."""
    return (i * n_poses) // steps if steps <= n_poses else i % n_poses


def timed_poses(steps, n_poses):
    """Description of the poses a run of `steps` frames times."""
    idx = sorted({pose_index(i, steps, n_poses) for i in range(steps)})
    if len(idx) == n_poses:
        return dict(poses=n_poses, pose_indices=f"all {n_poses} poses" + (", wrapping" if steps > n_poses else ""))
    stride = idx[1] - idx[0] if len(idx) > 1 else 0
    even = all(idx[j + 1] - idx[j] == stride for j in range(len(idx) - 1))
    desc = (f"{idx[0]}, {idx[1]}, ..., {idx[-1]} (every {stride}th of {n_poses})" if even and len(idx) > 2 else
            ", ".join(str(x) for x in idx[:8]) + (" ..." if len(idx) > 8 else "") + f" of {n_poses}")
    return dict(poses=len(idx), pose_indices=desc)


def run_variant(ctx, tigas, scene, storage, traj, k, W, H, steps, warmup, torch, count_work, tile_kw):
    s = ctx.load_scene(scene, storage)
    out = torch.empty((H, W, 3), dtype=torch.uint8, device="cuda")
    # warm-up: the first frame of this shape runs the autotuner and captures the graph
    for i in range(warmup):
        ctx.render(s, traj[i % len(traj)], k, W, H, out=out, **tile_kw)
    torch.cuda.synchronize()

    def timed(label):
        lat = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            t = time.perf_counter()
            ctx.render(s, traj[pose_index(i, steps, len(traj))], k, W, H, out=out, **tile_kw)
            lat.append(time.perf_counter() - t)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        p50, p99 = _stats(lat)
        return dict(frames_per_s=steps / total, ms_per_frame=1e3 * total / steps, p50_ms=p50, p99_ms=p99)

    # headline: the product path (graph replay per frame), no instrumentation
    head = timed("graph")
    cfg = ctx.stats()
    # the same frames submitted asynchronously (the next frame is launched
    # while the previous one renders; frames still run one after the other)
    outs = [out, torch.empty_like(out)]
    res, prev = [], None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        t = ctx.render_async(s, traj[pose_index(i, steps, len(traj))], k, W, H, outs[i % 2], **tile_kw)
        if prev is not None:
            res.append(ctx.wait(prev))
        prev = t
    res.append(ctx.wait(prev))
    total = time.perf_counter() - t0
    g = np.array([r["gpu_ms"] for r in res])
    pipelined = dict(frames_per_s=steps / total, gpu_ms_p50=float(np.median(g)), gpu_ms_p99=float(np.percentile(g, 99)),
                     gpu_ms_mean=float(g.mean()))
    # and on two streams (each with its own workspace): consecutive frames of
    # the trajectory run concurrently, one frame's latency-bound sort launches
    # beside the other's blend
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs2 = [out, outs[1]]
    for j, st in enumerate(streams):  # warm each stream's workspace and graph
        ctx.render(s, traj[0], k, W, H, out=outs2[j], stream=st.cuda_stream, **tile_kw)
    torch.cuda.synchronize()
    pend = []
    t0 = time.perf_counter()
    for i in range(steps):
        j = i % 2
        pend.append(ctx.render_async(s, traj[pose_index(i, steps, len(traj))], k, W, H, outs2[j],
                                     stream=streams[j].cuda_stream, **tile_kw))
        if len(pend) > 2:
            ctx.wait(pend.pop(0))
    for t in pend:
        ctx.wait(t)
    torch.cuda.synchronize()
    pipelined["two_streams_frames_per_s"] = steps / (time.perf_counter() - t0)
    # the same frames again with HIP events between the stages (uncaptured launches)
    ctx.profile_stages(True)
    prof = timed("stages")
    stages = ctx.stage_times()
    ctx.profile_stages(False)
    nfr = max(stages["frames"], 1)
    # and once more with HIP events around every kernel launch: per-kernel
    # average launch durations for the roofline
    ctx.profile_kernels(True)
    timed("kernels")
    kt = ctx.kernel_times()
    ctx.profile_kernels(False)
    kernels = {name: dict(launches_per_frame=l / steps, avg_us=1e3 * ms / max(l, 1), ms_per_frame=ms / steps)
               for name, (l, ms) in kt.items()}
    # algorithmic work of the same frames (untimed pass with the counting blend
    # kernel): visible Gaussians, duplicates, evaluations, contributions
    work = dict(frames=0, visible=0, duplicates=0, evaluations=0, contributions=0, fallbacks=0)
    if count_work:
        for i in range(steps):
            e, c = ctx.count_blend_work(s, traj[pose_index(i, steps, len(traj))], k, W, H,
                                        tile=(cfg["tile_w"], cfg["tile_h"]),
                                        batch_depth=cfg["batch_depth"], ppl=cfg["pixels_per_lane"])
            st = ctx.stats()
            work["frames"] += 1
            work["evaluations"] += e
            work["contributions"] += c
            for f in ("visible", "duplicates", "fallbacks"):
                work[f] += st[f]
    res = dict(head, pipelined=pipelined, tile=f"{cfg['tile_w']}x{cfg['tile_h']}", batch_depth=cfg["batch_depth"],
               sort_passes=cfg["sort_passes"],
               pixels_per_lane=cfg["pixels_per_lane"],
               stage_pass=prof, gpu_ms_per_frame=sum(v for kk, v in stages.items() if kk != "frames") / nfr,
               stage_ms={kk: v / nfr for kk, v in stages.items() if kk != "frames"},
               work=work, scene_bytes=s.bytes, kernels=kernels)
    s.free()
    return res


def run_plain(ctx, scene, traj, k, W, H, steps, warmup, torch):
    """The plain FP32 single-view renderer on another workload: frames/s and
    p50/p99 host latency per frame (graph replay, autotuned tile) over the
    same evenly spread poses, and the GPU time per frame (HIP events) of the
    same frames submitted asynchronously."""
    s = ctx.load_scene(scene, "f32")
    out = torch.empty((H, W, 3), dtype=torch.uint8, device="cuda")
    n = len(traj)
    for i in range(warmup):
        ctx.render(s, traj[i % n], k, W, H, out=out)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for i in range(steps):
        t = time.perf_counter()
        ctx.render(s, traj[pose_index(i, steps, n)], k, W, H, out=out)
        lat.append(time.perf_counter() - t)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    st = ctx.stats()
    outs = [out, torch.empty_like(out)]
    gms, prev = [], None
    for i in range(steps):
        t = ctx.render_async(s, traj[pose_index(i, steps, n)], k, W, H, outs[i % 2])
        if prev is not None:
            gms.append(ctx.wait(prev)["gpu_ms"])
        prev = t
    gms.append(ctx.wait(prev)["gpu_ms"])
    p50, p99 = _stats(lat)
    s.free()
    return dict(n_gaussians=scene.n, width=W, height=H, **timed_poses(steps, n), frames_per_s=steps / total,
                ms_per_frame=1e3 * total / steps, p50_ms=p50, p99_ms=p99, gpu_ms_mean=float(np.mean(gms)),
                tile=f"{st['tile_w']}x{st['tile_h']}", batch_depth=st["batch_depth"],
                pixels_per_lane=st["pixels_per_lane"], visible_last=st["visible"], duplicates_last=st["duplicates"])


def run_batched(ctx, scene, torch, steps=30, warmup=3):
    """The batched form: 32 poses of the trajectory at rungs 0.25/0.5/0.75/1.0
    of 1920x1080 (8 each) rendered as one step (one launch sequence with a
    persistent blend, replayed from a captured graph, autotuned tile / depth),
    against the same 32 views rendered one by one."""
    from paper_2605_08699_amd import synth
    poses, scales = synth.c4_views()
    k = synth.fov_intrinsics(1920, 1080)
    s = ctx.load_scene(scene, "f32")
    n = len(poses)
    outs = []
    for sc in scales:
        w, h = int(1920 * sc + 0.5), int(1080 * sc + 0.5)
        outs.append(torch.empty((h, w, 3), dtype=torch.uint8, device="cuda"))
    args = ([s] * n, poses, [k] * n, [1920] * n, [1080] * n, scales)
    for _ in range(warmup):
        ctx.render_batch(*args, outs=outs)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        t = time.perf_counter()
        ctx.render_batch(*args, outs=outs)
        lat.append(time.perf_counter() - t)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    st = ctx.stats()
    for i in range(n):  # one by one (graph replays of the single-view sequence)
        ctx.render(s, poses[i], k, 1920, 1080, res_scale=scales[i], out=outs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(3):
        for i in range(n):
            ctx.render(s, poses[i], k, 1920, 1080, res_scale=scales[i], out=outs[i])
    torch.cuda.synchronize()
    seq = (time.perf_counter() - t1) / 3
    p50, p99 = _stats(lat)
    px = sum(o.shape[0] * o.shape[1] for o in outs)
    s.free()
    return dict(views=n, megapixels_per_step=px / 1e6, step_ms_p50=p50, step_ms_p99=p99,
                views_per_s=n * steps / total, megapixels_per_s=px * steps / total / 1e6,
                sequential_views_per_s=n / seq, tile=f"{st['tile_w']}x{st['tile_h']}",
                batch_depth=st["batch_depth"], pixels_per_lane=st["pixels_per_lane"], duplicates=st["duplicates"],
                tiles=st["tiles"])


def run_jpeg(ctx, tigas, scene, traj, torch, steps=40):
    """The per-frame payload: each rung of the paper's bitrate ladder (Table 1:
    320x180 q10, 640x360 q35, 960x540 q65, 1280x720 q90, plus 1920x1080 q90)
    rendered from the 3M-Gaussian scene and encoded on the GPU.  Per rung:
    stream bytes, host time per encode call (launches + length read-back),
    per-kernel GPU times (HIP events), render + encode frames/s, and the JPEG
    oracle's single-thread time for the same frame."""
    from oracle import jpeg as oj
    from paper_2605_08699_amd import synth
    s = ctx.load_scene(scene, "f32")
    rungs = []
    for (w, h, q) in ((320, 180, 10), (640, 360, 35), (960, 540, 65), (1280, 720, 90), (1920, 1080, 90)):
        k = synth.fov_intrinsics(w, h)
        frame = torch.empty((h, w, 3), dtype=torch.uint8, device="cuda")
        out = torch.empty(int(tigas.lib().tigas_jpeg_max_bytes(w, h)), dtype=torch.uint8, device="cuda")
        for i in range(3):
            ctx.render(s, traj[i], k, w, h, out=frame)
            ctx.jpeg_encode(frame, q, out=out)
        torch.cuda.synchronize()
        sizes, enc = [], 0.0
        t0 = time.perf_counter()
        for i in range(steps):
            ctx.render(s, traj[i % len(traj)], k, w, h, out=frame)
            t = time.perf_counter()
            _, n = ctx.jpeg_encode(frame, q, out=out)
            enc += time.perf_counter() - t
            sizes.append(n)
        total = time.perf_counter() - t0
        ctx.profile_kernels(True)
        for _ in range(10):
            ctx.jpeg_encode(frame, q, out=out)
        kt = ctx.kernel_times()
        ctx.profile_kernels(False)
        kern = {n_: 1e3 * ms / l for n_, (l, ms) in kt.items() if "jpeg" in n_}
        img = frame.cpu().numpy()
        t = time.perf_counter()
        want = oj.encode(img, q)
        cpu_s = time.perf_counter() - t
        rungs.append(dict(width=w, height=h, quality=q, bytes_mean=float(np.mean(sizes)),
                          stream_equals_oracle=ctx.jpeg_bytes(frame, q) == want,
                          encode_ms=1e3 * enc / steps, kernel_us=kern, kernel_us_total=sum(kern.values()),
                          render_encode_frames_per_s=steps / total,
                          cpu_oracle_encode_ms=1e3 * cpu_s))
    s.free()
    return dict(rungs=rungs, cpu_oracle_threads=1)


def run_abr_clients(ctx, torch, tigas, serving_scenes, seconds=4.0, n_clients=16):
    """Closed-loop clients on the serving loop, each driven by the library's
    latency ABR (Section 5.3): a client sends its next request when it has
    received the previous payload, at the ladder level the ABR picked (Table
    1: 1280x720 scaled by 0.25/0.5/0.75/1 at JPEG quality 10/35/65/90); the
    server renders and encodes it; the payload then takes a simulated
    download: bytes / bandwidth + one RTT, the bandwidth a per-client mean
    (log-uniform 2..200 Mbit/s, seeded) times a log-normal factor per request.
    Rapid panning (rotation above 90 deg/s between requests) allows immediate
    downgrades.  Reports levels, latency (server + network) and switches."""
    from paper_2605_08699_amd import synth
    scenes = [ctx.load_scene(sc, "f16") for sc in serving_scenes]
    ladder = ((0.25, 10), (0.5, 35), (0.75, 65), (1.0, 90))
    k = synth.fov_intrinsics(1280, 720)
    rng = np.random.default_rng(4000)
    mean_bw = np.exp(rng.uniform(np.log(2e6), np.log(200e6), n_clients))  # bit/s
    rtt = rng.uniform(0.01, 0.06, n_clients)
    clients = synth.serving_clients(n_clients, rate_hz=60.0, duration_s=seconds + 2)
    frames = [torch.empty((720, 1280, 3), dtype=torch.uint8, device="cuda") for _ in range(n_clients)]
    jpegs = [torch.empty(8 << 20, dtype=torch.uint8, device="cuda") for _ in range(n_clients)]
    abrs = [tigas.ABR() for _ in range(n_clients)]
    level = [0] * n_clients
    step = [0] * n_clients
    next_send = [0.0] * n_clients
    inflight = {}
    recs = []
    with tigas.Server(ctx, slots=2, max_batch=64, hbm_budget=48 << 30) as sv:
        t0 = time.perf_counter()
        while True:
            now = time.perf_counter() - t0
            if now > seconds and not inflight:
                break
            for c in range(n_clients):
                if now >= next_send[c] and c not in [v[0] for v in inflight.values()] and now <= seconds:
                    cl = clients[c]
                    pose = cl.poses[min(step[c], len(cl.poses) - 1)]
                    sc, q = ladder[level[c]]
                    rid = sv.submit(tigas.request_c(scenes[cl.scene_id], pose, k, 1280, 720, frames[c], client=c,
                                                    res_scale=sc, jpeg_quality=q, jpeg_out=jpegs[c]))
                    inflight[rid] = (c, now, level[c], step[c])
            for d in sv.poll():
                c, sent, lv, st_ = inflight.pop(d["id"])
                server_s = d["done_s"] - d["arrival_s"]
                bw = mean_bw[c] * float(np.exp(rng.normal(0, 0.3)))
                dl = d["jpeg_bytes"] * 8.0 / bw
                total = server_s + rtt[c] + dl
                # rotation between this pose and the next: degrees per second of the walk
                cl = clients[c]
                p0, p1 = cl.poses[min(st_, len(cl.poses) - 1)], cl.poses[min(st_ + 1, len(cl.poses) - 1)]
                cosang = np.clip((np.trace(p0.R.T @ p1.R) - 1) / 2, -1, 1)
                pan = math.degrees(math.acos(cosang)) / max(total, 1e-3) > 90.0
                level[c] = abrs[c].observe(d["jpeg_bytes"], dl, pan)
                step[c] = st_ + 1
                next_send[c] = (time.perf_counter() - t0) + rtt[c] + dl  # the frame arrives, the next request leaves
                recs.append((c, lv, server_s, total, d["jpeg_bytes"], level[c] != lv))
            time.sleep(0.0002)
    for a in abrs:
        a.close()
    for s_ in scenes:
        s_.free()
    tot = np.array([r[3] for r in recs]) * 1e3
    srv = np.array([r[2] for r in recs]) * 1e3
    lv = np.array([r[1] for r in recs])
    return dict(clients=n_clients, seconds=seconds, requests=len(recs),
                level_share={str(l): float((lv == l).mean()) for l in range(4)},
                latency_ms_p50=float(np.median(tot)), latency_ms_p99=float(np.percentile(tot, 99)),
                within_100ms=float((tot <= 100.0).mean()), server_ms_p50=float(np.median(srv)),
                server_ms_p99=float(np.percentile(srv, 99)), mean_payload_bytes=float(np.mean([r[4] for r in recs])),
                switches_per_client=sum(r[5] for r in recs) / n_clients,
                bandwidth_mbps=[round(float(b) / 1e6, 1) for b in mean_bw])


def run_serving(ctx, torch, tigas, serving_scenes, seconds=10.0, warm=1.0, sweep_seconds=4.0,
                rates=(30.0, 40.0, 45.0, 50.0), budget_gb=48, batch_mpx=6.0, slots=2):
    """The serving form: 64 clients (Poisson arrivals, random rungs of
    1920x1080, their own 6DoF walks) on 4 resident FP16 scenes of 0.5/1/3/6M
    Gaussians, replayed open-loop into the library's continuous-batching
    server (memory budget).  Full offered load (60 req/s per client) for
    `seconds` after `warm` seconds of warm-up, with latest-pose-wins; then a
    shorter rate sweep without supersession for the largest per-client rate
    whose p99 latency for 1080p frames of the 3M scene stays within 10 ms;
    then full load and 40 req/s per client again with each frame also encoded
    as its JPEG payload.  A superseded request is not rendered: its client
    sees the frame of the request that replaced it, so besides the latency of
    rendered requests the report gives a p99 that counts each superseded
    request from its own arrival to that frame's completion."""
    from paper_2605_08699_amd import synth
    scenes = [ctx.load_scene(sc, "f16") for sc in serving_scenes]
    k = synth.fov_intrinsics(1920, 1080)
    outs = [torch.empty((1080, 1920, 3), dtype=torch.uint8, device="cuda") for _ in range(64)]
    jpeg_outs = [torch.empty(8 << 20, dtype=torch.uint8, device="cuda") for _ in range(64)]
    ladder_q = {0.25: 10, 0.5: 35, 0.75: 65, 1.0: 90}

    def trace(rate, duration, jpeg=False):
        clients = synth.serving_clients(64, rate_hz=rate, duration_s=duration)
        reqs = []
        for c, cl in enumerate(clients):
            for j in range(len(cl.arrivals_s)):
                reqs.append((cl.arrivals_s[j], c, cl.scene_id, cl.poses[j], float(cl.rungs[j])))
        reqs.sort(key=lambda r: r[0])
        cs = [tigas.request_c(scenes[sid], pose, k, 1920, 1080, outs[c], client=c, arrival_s=t, res_scale=rung,
                              jpeg_quality=ladder_q[rung] if jpeg else 0, jpeg_out=jpeg_outs[c] if jpeg else None)
              for t, c, sid, pose, rung in reqs]
        return cs, reqs

    def run(rate, supersede, measured, jpeg=False):
        cs, reqs = trace(rate, warm + measured, jpeg)
        with tigas.Server(ctx, slots=slots, max_batch=64, hbm_budget=int(budget_gb * 2 ** 30), supersede=supersede,
                          max_batch_pixels=int(batch_mpx * 1e6)) as sv:
            done = sv.replay(cs)
            st = sv.stats()
        lat, lat_hd, lat_all, lat_all_hd = [], [], [], []
        # completion of the next rendered request of each client, for the superseded ones
        next_done = {}
        served_by = [None] * len(done)
        for i in range(len(done) - 1, -1, -1):
            c = reqs[i][1]
            if done[i]["status"] == 0:
                next_done[c] = done[i]["done_s"]
            served_by[i] = next_done.get(c)
        for d, r, sb in zip(done, reqs, served_by):
            if r[0] < warm:
                continue
            hd = r[2] == 2 and r[4] == 1.0
            if d["status"] == 0:
                ms = 1e3 * (d["done_s"] - d["arrival_s"])
                lat.append(ms)
                lat_all.append(ms)
                if hd:
                    lat_hd.append(ms)
                    lat_all_hd.append(ms)
            elif d["status"] == 1 and sb is not None:
                ms = 1e3 * (sb - d["arrival_s"])
                lat_all.append(ms)
                if hd:
                    lat_all_hd.append(ms)
        rendered = sum(1 for d, r in zip(done, reqs) if d["status"] == 0 and r[0] >= warm)
        jb = [d["jpeg_bytes"] for d, r in zip(done, reqs) if d["status"] == 0 and r[0] >= warm and jpeg]
        pct = lambda a, q: float(np.percentile(a, q)) if a else None
        return dict(rate_per_client=rate, measured_s=measured, warmup_s=warm, supersede=supersede,
                    offered_req_per_s=sum(1 for r in reqs if r[0] >= warm) / measured,
                    rendered_frames_per_s=rendered / measured, p50_ms=pct(lat, 50), p99_ms=pct(lat, 99),
                    p50_ms_1080p_3M=pct(lat_hd, 50), p99_ms_1080p_3M=pct(lat_hd, 99),
                    p99_ms_counting_superseded=pct(lat_all, 99),
                    p99_ms_1080p_3M_counting_superseded=pct(lat_all_hd, 99),
                    superseded=st["superseded"], deferred=st["deferred"], admitted=st["admitted"],
                    batches=st["batches"], mean_batch=st["admitted"] / max(st["batches"], 1), failed=st["failed"],
                    jpeg_mean_bytes=float(np.mean(jb)) if jb else None,
                    jpeg_over_capacity=sum(1 for b in jb if b > (8 << 20)))

    full = run(60.0, True, seconds)
    sweep = [run(r, False, sweep_seconds) for r in rates]
    # the same with the per-request payload: every frame also encoded as the
    # JPEG of its rung's quality (Table 1), done when the payload is
    full_jpeg = run(60.0, True, seconds, jpeg=True)
    at40_jpeg = run(40.0, False, sweep_seconds, jpeg=True)
    ok = [x["rate_per_client"] for x in sweep if x["p99_ms_1080p_3M"] is not None and x["p99_ms_1080p_3M"] <= 10.0]
    for s_ in scenes:
        s_.free()
    return dict(seconds=seconds, warmup_s=warm, clients=64, hbm_budget_gb=budget_gb, slots=slots,
                max_batch_megapixels=batch_mpx,
                full_load_latest_pose_wins=full, sweep_no_supersede=sweep,
                with_jpeg={"full_load_latest_pose_wins": full_jpeg, "rate_40_no_supersede": at40_jpeg,
                           "quality_by_rung": {str(k_): v for k_, v in ladder_q.items()}},
                max_rate_per_client_p99_1080p_3M_within_10ms=max(ok) if ok else None)


def kernel_work(name, w, n, storage, tile_passes):
    """Algorithmic work of a kernel per FRAME (all its launches of the frame),
    averaged over the frames of the work pass: (bound, amount) with bytes for
    HBM-bound kernels and FP32 flops for the blend, or None for a kernel
    without a model."""
    nf = max(w["frames"], 1)
    D = w["duplicates"] / nf
    V = w["visible"] / nf
    if "k_blend" in name:
        return "alu", (FLOPS_EVAL * w["evaluations"] + FLOPS_CONTRIB * w["contributions"]) / nf
    if "k_preprocess" in name:
        # attributes of every Gaussian, SH of the visible ones, depth key +
        # tile rectangle of every record, one 64-byte record per visible
        attr = 44 if storage == "f32" else 28
        shb = 192 if storage == "f32" else 96
        return "hbm", n * attr + V * shb + n * 12 + V * 64
    if "k_duplicate" in name:
        # sorted record id and packed tile rectangle per visible Gaussian;
        # tile word + record id per duplicate
        return "hbm", V * 8 + D * 8
    if "k_sort_downsweep<true, false, " in name:
        # the depth passes (three of 9-bit digits, else four of 8 bits): key,
        # record and packed rectangle read and written
        return "hbm", (3 if "false, 512" in name else 4) * 24 * V
    if "k_sort_downsweep<false, false, " in name:
        # the tile passes: key + value read and written per duplicate
        return "hbm", tile_passes * 16 * D
    if "k_bin_emit" in name:
        # depth-ordered record and packed rectangle read per visible Gaussian,
        # one record id written per entry
        return "hbm", V * 8 + D * 4
    return None


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_3M_1080p_f32.md")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter profile, or
    None when it was measured on other kernel source (or not at all)."""
    from paper_2605_08699_amd import profiling
    sha, t = profiling.read_traffic(TRAFFIC_FILE)
    if sha != profiling.source_sha1():
        return None
    return t.get(kernel)


def roofline(v, n, storage):
    """Roofline of the dominant kernel of the FP32 run: algorithmic work per
    launch / average launch duration (HIP events around every launch)."""
    w = v["work"]
    depth_passes = 3 if any("k_sort_downsweep<true, false, 512" in k for k in v["kernels"]) else 4
    tile_passes = v["sort_passes"] - depth_passes
    ranked = sorted(v["kernels"].items(), key=lambda kv: -kv[1]["ms_per_frame"])
    for name, k in ranked:
        m = kernel_work(name, w, n, storage, tile_passes)
        if m is None:
            continue
        bound, amount = m
        amount /= max(k["launches_per_frame"], 1e-9)
        sec = k["avg_us"] * 1e-6
        traffic = measured_traffic(name)
        if bound == "alu":
            ach = amount / sec / 1e12
            # the survey's cost model: 15 VALU operations + 1 exp per evaluation
            evals = w["evaluations"] / max(w["frames"], 1) / max(k["launches_per_frame"], 1e-9)
            ach16 = OPS_EVAL_MODEL * evals / sec / 1e12
            return dict(kernel=name, bound="alu", achieved=ach, peak=FP32_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                        frac=ach / FP32_VECTOR_PEAK_TFLOPS, traffic=traffic, avg_us=k["avg_us"],
                        per_launch=amount, dominant=ranked[0][0], evaluations_per_launch=evals,
                        achieved_16_ops_per_evaluation=ach16, frac_16_ops_per_evaluation=ach16 / FP32_VECTOR_PEAK_TFLOPS)
        ach = amount / sec / 1e9
        return dict(kernel=name, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                    traffic=traffic, avg_us=k["avg_us"], per_launch=amount, dominant=ranked[0][0])
    return None


def hbm_copy(torch, mib=1024, reps=20):
    """A plain device-to-device copy of known size (torch's elementwise copy
    kernel): the achievable HBM rate, and the reference that scales profiler
    byte counters (FETCH_SIZE / WRITE_SIZE) into bytes."""
    n = mib * 2 ** 20 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) * 1e-3 / reps
    moved = 2 * n * 4
    del src, dst
    return dict(bytes_read=n * 4, bytes_written=n * 4, us=sec * 1e6, gbps=moved / sec / 1e9)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_frame_s(orc, scene, pose, k, W, H, n_pix, seed=0):
    """Seconds of one full frame of the FP64 oracle, extrapolated from the
    projection + depth order of every Gaussian and n_pix random pixels."""
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    proj = orc.preprocess(scene, pose, k, W, H)
    _ = proj.order
    proj.boxes()
    t1 = time.perf_counter()
    if n_pix >= W * H:
        yy, xx = np.mgrid[0:H, 0:W]
        orc.render_pixels(proj, xx.reshape(-1), yy.reshape(-1))
        n_pix = W * H
    else:
        idx = rng.choice(W * H, n_pix, replace=False)
        orc.render_pixels(proj, idx % W, idx // W)
    t2 = time.perf_counter()
    return (t1 - t0) + (t2 - t1) * (W * H / n_pix), t1 - t0, t2 - t1


def cpu_baseline(scene, pose, k, W, H, c1=None, n_pix=100_000, n_pix_1t=8_000):
    """The FP64 oracle, untuned, on bounded samples: the headline frame (pose
    0 of the 3M-Gaussian 1080p trajectory) on all host threads and on one
    thread, and the full 20k-Gaussian 256x256 frame on all threads."""
    from oracle import oracle as orc
    threads = orc.num_threads()
    frame_s, proj_s, pix_s = _oracle_frame_s(orc, scene, pose, k, W, H, n_pix)
    orc.set_threads(1)
    try:
        frame_1t, proj_1t, pix_1t = _oracle_frame_s(orc, scene, pose, k, W, H, n_pix_1t, seed=1)
    finally:
        orc.set_threads(threads)
    res = dict(value=1.0 / frame_s, unit="frames/s", cores=threads, kind="oracle", cpu_model=cpu_model(),
               sample=f"pose 0 of the {scene.n}-Gaussian {W}x{H} trajectory: FP64 projection + depth order of every "
                      f"Gaussian ({proj_s:.2f} s) and {n_pix} random pixels ({pix_s:.2f} s) on {threads} threads, "
                      f"extrapolated to the full frame",
               seconds_per_frame=frame_s,
               one_thread={"value": 1.0 / frame_1t, "unit": "frames/s", "seconds_per_frame": frame_1t,
                           "sample": f"the same frame on 1 thread: projection {proj_1t:.2f} s, {n_pix_1t} random "
                                     f"pixels {pix_1t:.2f} s, extrapolated"})
    if c1 is not None:
        sc1, p1, k1, W1, H1 = c1
        f1, _, _ = _oracle_frame_s(orc, sc1, p1, k1, W1, H1, W1 * H1)
        res["c1_full_frame"] = {"seconds_per_frame": f1, "frames_per_s": 1.0 / f1, "threads": threads,
                                "sample": f"every pixel of the {sc1.n}-Gaussian {W1}x{H1} frame"}
    return res


def run_registry(ctx, tigas, synth):
    """Model registry: the first access of a model (PLY parse + upload into the
    resident layout) against a re-acquire of the resident model, for the
    1M-Gaussian SH-degree-3 scene written as a binary 3DGS PLY.  The file sits
    in the host's page cache (written just before), so the parse is measured
    without disk reads."""
    import shutil
    import tempfile
    d = tempfile.mkdtemp(prefix="tigas_models_")
    try:
        sc = synth.c2_scene()
        os.makedirs(os.path.join(d, "c2"))
        path = os.path.join(d, "c2", "point_cloud.ply")
        synth.write_ply(path, sc)
        size = os.path.getsize(path)
        t0 = time.perf_counter()
        tigas.ply_read(path)
        parse_s = time.perf_counter() - t0
        reg = tigas.Registry(ctx, d, idle_timeout_s=0.0)
        try:
            t0 = time.perf_counter()
            s1 = reg.acquire("c2")
            cold_s = time.perf_counter() - t0
            warm = []
            for _ in range(20):
                t0 = time.perf_counter()
                s2 = reg.acquire("c2")
                warm.append(time.perf_counter() - t0)
                reg.release(s2)
            resident = reg.info("c2")["device_bytes"]
            reg.release(s1)
            t0 = time.perf_counter()
            ev = reg.evict_idle()
            evict_s = time.perf_counter() - t0
        finally:
            reg.close()
        return dict(model="1M Gaussians, SH degree 3, binary little-endian 3DGS PLY", file_bytes=size,
                    resident_bytes=resident, parse_ms=1e3 * parse_s, parse_gb_per_s=size / parse_s / 1e9,
                    first_access_ms=1e3 * cold_s, resident_acquire_us=1e6 * float(np.median(warm)),
                    evicted=ev, evict_ms=1e3 * evict_s)
    finally:
        shutil.rmtree(d, ignore_errors=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=3_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", default="f32,f16,bf16")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the 20k/256x256 and 1M/1280x720 renderer runs")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-jpeg", action="store_true")
    ap.add_argument("--no-abr", action="store_true")
    ap.add_argument("--no-registry", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="measured seconds of each full-load serving run (after 1 s of warm-up)")
    ap.add_argument("--tile", default=None,
                    help="W,H,batch_depth,pixels_per_lane for the single-view variants (default: autotuned)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py renders on one GPU only: the rasterizer has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_08699_amd import synth, tigas

    W, H = 1920, 1080
    scene = synth.c3_scene(args.n)
    traj = synth.c3_trajectory(300)
    k = synth.fov_intrinsics(W, H)
    ctx = tigas.Context(0)
    copy = hbm_copy(torch)
    print(f"# HBM copy: {copy['gbps']:.0f} GB/s", file=sys.stderr, flush=True)
    variants = {}
    for storage in args.variants.split(","):
        tile_kw = {}
        if args.tile:
            tw, th, bd, ppl = (int(x) for x in args.tile.split(","))
            tile_kw = dict(tile=(tw, th), batch_depth=bd, ppl=ppl)
        variants[storage] = run_variant(ctx, tigas, scene, storage, traj, k, W, H, args.steps, args.warmup, torch,
                                        count_work=(storage == "f32"), tile_kw=tile_kw)
        print(f"# {storage}: {variants[storage]['frames_per_s']:.1f} frames/s, p50 "
              f"{variants[storage]['p50_ms']:.3f} ms, p99 {variants[storage]['p99_ms']:.3f} ms", file=sys.stderr,
              flush=True)
    main_v = variants["f32"] if "f32" in variants else next(iter(variants.values()))
    rl = roofline(main_v, scene.n, "f32")
    line = {
        "metric": "frames/s + p50/p99 render latency, 3M Gaussians @1080p, fp32 vs fp16-attr",
        "value": main_v["frames_per_s"],
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_v["ms_per_frame"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3M Gaussians (64 clusters + 40% surface splats, SH deg 3), 1920x1080, "
                               "300-pose 6DoF trajectory, FP32 attributes, RGB8 frame in HBM",
                   "n_gaussians": scene.n, "width": W, "height": H, "trajectory_poses": len(traj),
                   **timed_poses(args.steps, len(traj)),
                   "tile": main_v["tile"], "batch_depth": main_v["batch_depth"],
                   "pixels_per_lane": main_v["pixels_per_lane"]},
        "p50_ms": main_v["p50_ms"],
        "p99_ms": main_v["p99_ms"],
        "gpu_ms_per_frame": main_v["gpu_ms_per_frame"],
        "stage_ms": main_v["stage_ms"],
        "work_per_frame": {x: main_v["work"][x] / max(main_v["work"]["frames"], 1)
                           for x in ("visible", "duplicates", "evaluations", "contributions", "fallbacks")},
        "stage_pass": main_v["stage_pass"],
        "pipelined": main_v["pipelined"],
        "variants": {kk: {x: vv[x] for x in ("frames_per_s", "p50_ms", "p99_ms", "gpu_ms_per_frame", "stage_ms",
                                              "scene_bytes", "tile", "batch_depth", "pixels_per_lane", "pipelined")}
                     for kk, vv in variants.items()},
        "roofline": {x: rl[x] for x in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_kernel": {x: rl[x] for x in ("kernel", "avg_us", "per_launch", "dominant", "evaluations_per_launch",
                                               "achieved_16_ops_per_evaluation", "frac_16_ops_per_evaluation")
                            if x in rl},
        "hbm_copy": copy,
        "kernels": main_v["kernels"],
    }
    if not args.no_plain:
        # the plain FP32 renderer on the two smaller workloads, same steps
        c1s, c1p, c1k, c1w, c1h = synth.c1_single_view()
        line["plain_20k_256"] = run_plain(ctx, c1s, c1p, c1k, c1w, c1h, args.steps, args.warmup, torch)
        line["plain_1M_720p"] = run_plain(ctx, synth.c2_scene(), synth.c2_trajectory(300),
                                          synth.fov_intrinsics(1280, 720), 1280, 720, args.steps, args.warmup, torch)
        for key in ("plain_20k_256", "plain_1M_720p"):
            p = line[key]
            print(f"# {key}: {p['frames_per_s']:.0f} frames/s, p50 {p['p50_ms']:.3f} ms, p99 {p['p99_ms']:.3f} ms",
                  file=sys.stderr, flush=True)
    if not args.no_batched:
        line["batched"] = run_batched(ctx, scene, torch)
        print(f"# batched: {line['batched']['views_per_s']:.0f} views/s "
              f"(one by one: {line['batched']['sequential_views_per_s']:.0f})", file=sys.stderr, flush=True)
    if not args.no_jpeg:
        line["jpeg"] = run_jpeg(ctx, tigas, scene, traj, torch)
        r = line["jpeg"]["rungs"][3]
        print(f"# jpeg 1280x720 q90: {r['bytes_mean'] / 1024:.0f} KiB, encode {r['encode_ms']:.3f} ms per call, "
              f"render+encode {r['render_encode_frames_per_s']:.0f} frames/s", file=sys.stderr, flush=True)
    serving_scenes = synth.serving_scenes() if not (args.no_serving and args.no_abr) else None
    if not args.no_serving:
        line["serving"] = run_serving(ctx, torch, tigas, serving_scenes, seconds=args.serve_seconds)
        f = line["serving"]["full_load_latest_pose_wins"]
        print(f"# serving at {f['offered_req_per_s']:.0f} req/s offered: {f['rendered_frames_per_s']:.0f} frames/s, "
              f"p50 {f['p50_ms']:.2f} ms p99 {f['p99_ms']:.2f} ms (1080p 3M: p99 {f['p99_ms_1080p_3M']})",
              file=sys.stderr, flush=True)
        j = line["serving"]["with_jpeg"]["rate_40_no_supersede"]
        print(f"# serving with JPEG payloads at 40 req/s per client: {j['rendered_frames_per_s']:.0f} frames/s, "
              f"p99 {j['p99_ms']:.2f} ms (1080p 3M: p99 {j['p99_ms_1080p_3M']}), mean {j['jpeg_mean_bytes']:.0f} B",
              file=sys.stderr, flush=True)
    if not args.no_abr:
        line["abr_clients"] = run_abr_clients(ctx, torch, tigas, serving_scenes)
        a = line["abr_clients"]
        print(f"# ABR clients: {a['requests']} requests, levels {a['level_share']}, latency p50 "
              f"{a['latency_ms_p50']:.1f} ms p99 {a['latency_ms_p99']:.1f} ms, {100 * a['within_100ms']:.0f}% "
              f"within 100 ms", file=sys.stderr, flush=True)
    if not args.no_registry:
        line["registry"] = run_registry(ctx, tigas, synth)
        g = line["registry"]
        print(f"# registry: first access {g['first_access_ms']:.0f} ms ({g['file_bytes'] / 1e6:.0f} MB PLY, parse "
              f"{g['parse_ms']:.0f} ms), resident acquire {g['resident_acquire_us']:.1f} us", file=sys.stderr,
              flush=True)
    if not args.no_cpu_baseline:
        c1s, c1p, c1k, c1w, c1h = synth.c1_single_view()
        line["cpu_baseline"] = cpu_baseline(scene, traj[0], k, W, H, c1=(c1s, c1p[0], c1k, c1w, c1h))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
