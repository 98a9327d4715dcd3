"""Serving form (needs an MI355X): continuous batching of client requests
under a memory budget.  Every rendered frame must be identical to rendering
the request alone, and served frames match the FP64 oracle on sampled
pixels."""
import numpy as np
import pytest
import torch

from oracle import jpeg as oj
from oracle import oracle as orc
from paper_2605_08699_amd import synth, tigas
from tests import gpu_checks as gc
from tests.handmade import random_tiny_scene

pytestmark = pytest.mark.gpu

W, H = 640, 360


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = tigas.Context(0)
    yield c
    c.close()


SOURCES = {}  # loaded scene handle -> the attributes as the library stores them (for the oracle)


@pytest.fixture(scope="module")
def scenes(ctx):
    srcs = [(synth.c2_scene(150_000), "f32"),
            (random_tiny_scene(np.random.default_rng(9), n=8000, extent=3.0, depth=(2.0, 9.0)), "f16"),
            (synth.scene_clusters(seed=61, n=60_000, n_clusters=8, surface_frac=0.4), "bf16")]
    loaded = []
    for sc, storage in srcs:
        h = ctx.load_scene(sc, storage)
        SOURCES[id(h)] = sc if storage == "f32" else gc.round_attrs(sc, storage)
        loaded.append(h)
    yield loaded
    for s in loaded:
        s.free()


def _requests(scenes, n, seed):
    rng = np.random.default_rng(seed)
    traj = synth.trajectory(seed=seed, n_poses=n)
    k = synth.fov_intrinsics(W, H)
    reqs, outs, meta = [], [], []
    for i in range(n):
        sc = scenes[int(rng.integers(0, len(scenes)))]
        rung = float(rng.choice(synth.RUNG_SCALES))
        ow, oh = tigas.output_size(W, H, rung)
        out = np.zeros((oh, ow, 3), np.float32)
        reqs.append(tigas.request_c(sc, traj[i], k, W, H, out, client=i % 5, res_scale=rung, fmt="f32"))
        outs.append(out)
        meta.append((sc, traj[i], k, rung))
    return reqs, outs, meta


def _alone(ctx, meta):
    sc, pose, k, rung = meta
    return ctx.render(sc, pose, k, W, H, res_scale=rung, fmt="f32", tile=(16, 32), batch_depth=64)


def test_results_identical_alone_and_in_the_mix(ctx, scenes):
    reqs, outs, meta = _requests(scenes, 40, seed=21)
    with tigas.Server(ctx, slots=2, max_batch=16) as sv:
        for r in reqs:
            sv.submit(r)
        sv.drain()
        done = sv.poll()
        st = sv.stats()
    _say("mix", st)
    assert len(done) == 40 and all(d["status"] == 0 for d in done)
    assert st["batches"] < 40 and st["max_batch_seen"] > 1      # requests were batched together
    rng = np.random.default_rng(3)
    for i in range(40):
        np.testing.assert_array_equal(outs[i], _alone(ctx, meta[i]), err_msg=f"request {i}")
        # and each served frame against the FP64 oracle on sampled pixels
        sc, pose, k, rung = meta[i]
        proj = orc.preprocess(SOURCES[id(sc)], pose, k, W, H, scale=rung)
        idx = rng.choice(proj.out_w * proj.out_h, 200, replace=False)
        px, py = idx % proj.out_w, idx // proj.out_w
        br, nb = orc.render_pixels(proj, px, py)
        res = gc.check_frame_pixels(outs[i][py, px], br, nb)
        assert res["n_bad"] == 0 and res["n_unresolved"] == 0, (i, res)


def test_jpeg_payloads_in_the_mix(ctx, scenes):
    # RGB8 frames in device memory, each encoded as its request's JPEG at the
    # quality of its rung (the ladder pairs 10/35/65/90 with rising size)
    quality = {0.25: 10, 0.5: 35, 0.75: 65, 1.0: 90}
    rng = np.random.default_rng(31)
    traj = synth.trajectory(seed=31, n_poses=24)
    k = synth.fov_intrinsics(W, H)
    reqs, frames, jpegs, meta = [], [], [], []
    for i in range(24):
        sc = scenes[int(rng.integers(0, len(scenes)))]
        rung = float(rng.choice(synth.RUNG_SCALES))
        ow, oh = tigas.output_size(W, H, rung)
        frame = torch.zeros((oh, ow, 3), dtype=torch.uint8, device="cuda")
        jpeg = torch.zeros(int(tigas.lib().tigas_jpeg_max_bytes(ow, oh)), dtype=torch.uint8, device="cuda")
        reqs.append(tigas.request_c(sc, traj[i], k, W, H, frame, client=i % 6, res_scale=rung,
                                    jpeg_quality=quality[rung], jpeg_out=jpeg))
        frames.append(frame)
        jpegs.append(jpeg)
        meta.append((sc, traj[i], rung))
    with tigas.Server(ctx, slots=2, max_batch=8) as sv:
        for r in reqs:
            sv.submit(r)
        sv.drain()
        done = {d["id"]: d for d in sv.poll()}
        st = sv.stats()
    _say("jpeg mix", st)
    assert len(done) == 24 and st["max_batch_seen"] > 1
    for i in range(24):
        d = done[i]
        assert d["status"] == 0 and d["jpeg_bytes"] > 0
        img = frames[i].cpu().numpy()
        sc, pose, rung = meta[i]
        alone = ctx.render(sc, pose, k, W, H, res_scale=rung, tile=(16, 32), batch_depth=64)
        np.testing.assert_array_equal(img, alone, err_msg=f"frame {i}")
        got = bytes(jpegs[i][:d["jpeg_bytes"]].cpu().numpy())
        assert got == oj.encode(img, quality[rung]), f"payload {i}"


def test_small_budget_defers_requests_but_renders_them_all(ctx, scenes):
    reqs, outs, meta = _requests(scenes, 20, seed=22)
    # room for about two requests of the largest scene per slot
    budget = 2 * 2 * (150_016 * 88 + 150_016 * 5 * 24) + (1 << 20)
    with tigas.Server(ctx, slots=2, max_batch=64, hbm_budget=budget) as sv:
        for r in reqs:
            sv.submit(r)
        sv.drain()
        done = sv.poll()
        st = sv.stats()
    _say("budget", st)
    assert len(done) == 20 and all(d["status"] == 0 for d in done)
    assert st["deferred"] > 0 and st["batches"] >= 3
    for i in range(20):
        np.testing.assert_array_equal(outs[i], _alone(ctx, meta[i]), err_msg=f"request {i}")


def test_request_over_the_whole_budget_is_refused(ctx, scenes):
    reqs, outs, meta = _requests(scenes[:1], 1, seed=23)
    with tigas.Server(ctx, slots=1, hbm_budget=1 << 20) as sv:
        with pytest.raises(tigas.TigasError, match="E_BUDGET"):
            sv.submit(reqs[0])


def test_latest_pose_wins(ctx, scenes):
    k = synth.fov_intrinsics(W, H)
    traj = synth.trajectory(seed=24, n_poses=60)
    outs = [np.zeros((H, W, 3), np.uint8) for _ in range(60)]
    with tigas.Server(ctx, slots=1, max_batch=1, supersede=True) as sv:
        ids = [sv.submit(tigas.request_c(scenes[0], traj[i], k, W, H, outs[i], client=7)) for i in range(60)]
        sv.drain()
        done = {d["id"]: d for d in sv.poll()}
        st = sv.stats()
    _say("supersede", st)
    assert st["superseded"] > 0 and st["superseded"] + st["rendered"] == 60
    assert done[ids[-1]]["status"] == 0                       # the newest pose is always rendered
    last = ctx.render(scenes[0], traj[59], k, W, H, tile=(16, 32), batch_depth=64)
    np.testing.assert_array_equal(outs[59], last)


def test_open_loop_replay_reports_latencies(ctx, scenes):
    rng = np.random.default_rng(25)
    k = synth.fov_intrinsics(W, H)
    reqs, keep = [], []
    t = 0.0
    for i in range(120):
        t += rng.exponential(1 / 400.0)
        out = np.zeros((H, W, 3), np.uint8)
        keep.append(out)
        pose = synth.Pose(synth.look_at([0, 0, -8 + 0.01 * i]).astype(np.float32),
                          np.array([0, 0, -8 + 0.01 * i], np.float32))
        reqs.append(tigas.request_c(scenes[i % 3], pose, k, W, H, out, client=i % 8, arrival_s=t,
                                    res_scale=float(rng.choice(synth.RUNG_SCALES))))
    with tigas.Server(ctx, slots=2) as sv:
        done = sv.replay(reqs)
    lat = np.array([d["done_s"] - d["arrival_s"] for d in done])
    arr = np.array([d["arrival_s"] for d in done])
    _say("replay p50 %.3f ms p99 %.3f ms" % (1e3 * np.median(lat), 1e3 * np.percentile(lat, 99)))
    assert all(d["status"] == 0 for d in done)
    assert np.all(lat > 0) and np.all(np.diff(arr) >= 0)
    assert abs(arr[-1] - t) < 0.05
