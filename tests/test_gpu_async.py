"""Asynchronous frames (needs an MI355X): a frame is launched while the
previous one still renders; every frame must equal the synchronous render."""
import ctypes
import math

import numpy as np
import pytest
import torch

from paper_2605_08699_amd import synth, tigas
from tests.handmade import make_scene

pytestmark = pytest.mark.gpu

W, H = 1280, 720


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = tigas.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c2(ctx):
    s = ctx.load_scene(synth.c2_scene(1_000_000))
    yield s, synth.c2_trajectory(16), synth.fov_intrinsics(W, H)
    s.free()


def _outs(n=2):
    return [torch.empty((H, W, 3), dtype=torch.uint8, device="cuda") for _ in range(n)]


def test_pipelined_frames_equal_synchronous_renders(ctx, c2):
    s, traj, k = c2
    outs = _outs()
    got, stats = [], []
    prev = None
    for i in range(12):
        t = ctx.render_async(s, traj[i], k, W, H, outs[i % 2], tile=(16, 32), batch_depth=64)
        if prev is not None:
            stats.append(ctx.wait(prev))
            got.append(outs[(i - 1) % 2].cpu().numpy())
        prev = t
    stats.append(ctx.wait(prev))
    got.append(outs[11 % 2].cpu().numpy())
    _say("async stats", stats[-1])
    for i in range(12):
        want = ctx.render(s, traj[i], k, W, H, tile=(16, 32), batch_depth=64)
        np.testing.assert_array_equal(got[i], want, err_msg=f"frame {i}")
        assert stats[i]["gpu_ms"] > 0 and stats[i]["duplicates"] > 0


def test_third_submission_completes_the_oldest(ctx, c2):
    s, traj, k = c2
    outs = _outs(3)
    tickets = [ctx.render_async(s, traj[i], k, W, H, outs[i], tile=(16, 16), batch_depth=64) for i in range(3)]
    res = [ctx.wait(t) for t in tickets]
    for i in range(3):
        want = ctx.render(s, traj[i], k, W, H, tile=(16, 16), batch_depth=64)
        np.testing.assert_array_equal(outs[i].cpu().numpy(), want, err_msg=f"frame {i}")
        assert res[i]["tiles"] == 80 * 45
    with pytest.raises(tigas.TigasError, match="E_INVALID"):
        ctx.wait(tickets[0])  # collected already


def test_synchronous_call_between_async_frames(ctx, c2):
    s, traj, k = c2
    outs = _outs()
    t0 = ctx.render_async(s, traj[3], k, W, H, outs[0], tile=(16, 32), batch_depth=64)
    mid = ctx.render(s, traj[4], k, W, H, tile=(16, 32), batch_depth=64)
    t1 = ctx.render_async(s, traj[5], k, W, H, outs[1], tile=(16, 32), batch_depth=64)
    ctx.wait(t1)
    ctx.wait(t0)
    for o, i in ((outs[0], 3), (outs[1], 5)):
        np.testing.assert_array_equal(o.cpu().numpy(), ctx.render(s, traj[i], k, W, H, tile=(16, 32), batch_depth=64))
    np.testing.assert_array_equal(mid, ctx.render(s, traj[4], k, W, H, tile=(16, 32), batch_depth=64))


def test_overflowing_async_frame_is_rendered_again(ctx):
    # large splats: far more duplicates than the first workspace sizing allows
    rng = np.random.default_rng(7)
    n = 300_000
    means = np.stack([rng.uniform(-2, 2, n), rng.uniform(-1.2, 1.2, n), rng.uniform(4, 6, n)], 1)
    sc = make_scene(means, log_scales=np.full((n, 3), math.log(0.12)), logits=np.full(n, -3.0))
    other = tigas.Context(0)
    try:
        s = other.load_scene(sc)
        k = synth.fov_intrinsics(W, H)
        pose = synth.Pose(np.eye(3, dtype=np.float32), np.zeros(3, np.float32))
        out = _outs(1)[0]
        t = other.render_async(s, pose, k, W, H, out, tile=(16, 16), batch_depth=64)
        st = other.wait(t)
        _say("overflow async", st)
        assert st["rerenders"] >= 1 and st["duplicates"] > 4 * n
        np.testing.assert_array_equal(out.cpu().numpy(), other.render(s, pose, k, W, H, tile=(16, 16), batch_depth=64))
        s.free()
    finally:
        other.close()


def test_async_rejects_host_output_and_unknown_tickets(ctx, c2):
    s, traj, k = c2
    host = np.zeros((H, W, 3), np.uint8)
    fr = tigas.FrameC(ctypes.c_void_p(host.ctypes.data), host.nbytes, 0, 0, 0)
    q = tigas.quality_c(1.0, -1, "rgb8", (0, 0, 0), (16, 16), 64, None)
    t = ctypes.c_int64(0)
    rc = tigas.lib().tigas_render_submit(s.handle, ctypes.byref(tigas.pose_c(traj[0])), ctypes.byref(tigas.intr_c(k)),
                                         W, H, ctypes.byref(q), ctypes.byref(fr), None, ctypes.byref(t))
    assert rc == -1  # E_INVALID
    with pytest.raises(tigas.TigasError, match="E_INVALID"):
        ctx.wait(10 ** 12)
