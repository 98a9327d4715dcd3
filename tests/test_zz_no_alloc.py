"""The allocation-free render entry point (needs an MI355X): every frame it
enqueues equals the frame tigas_render gives for the same request and tile
configuration, call after call on the shared scratch array, including after
a call that overflowed the array's duplicate capacity."""
import numpy as np
import pytest
import torch

from paper_2605_08699_amd import synth, tigas

pytestmark = pytest.mark.gpu

TILE = dict(tile=(16, 16), batch_depth=64, ppl=1)


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = tigas.Context(0)
    yield c
    c.close()


def _noalloc(ctx, s, pose, k, w, h, fmt, res_scale=1.0, **kw):
    ow, oh = tigas.output_size(w, h, res_scale)
    out = torch.full((oh, ow, 3), 77, dtype=torch.uint8 if fmt == "rgb8" else torch.float32, device="cuda")
    cnt = torch.full((6,), -1, dtype=torch.int32, device="cuda")
    ctx.render_noalloc(s, pose, k, w, h, out, counters=cnt, res_scale=res_scale, fmt=fmt, **kw)
    torch.cuda.synchronize()
    c = cnt.cpu().numpy()
    return out, dict(duplicates=int(c[0]), visible=int(c[1]), fallbacks=int(c[2]), overflow=int(c[3]))


def _reference(ctx, s, pose, k, w, h, fmt, res_scale=1.0, **kw):
    ow, oh = tigas.output_size(w, h, res_scale)
    out = torch.empty((oh, ow, 3), dtype=torch.uint8 if fmt == "rgb8" else torch.float32, device="cuda")
    ctx.render(s, pose, k, w, h, out=out, res_scale=res_scale, fmt=fmt, **TILE, **kw)
    torch.cuda.synchronize()
    return out, ctx.stats()


def _same(ctx, s, pose, k, w, h, fmt, res_scale=1.0, **kw):
    got, c = _noalloc(ctx, s, pose, k, w, h, fmt, res_scale, **kw)
    want, st = _reference(ctx, s, pose, k, w, h, fmt, res_scale, **kw)
    _say(f"{w}x{h}@{res_scale} {fmt}: counters {c}, render stats D={st['duplicates']} V={st['visible']}")
    assert c["overflow"] == 0
    assert (c["duplicates"], c["visible"], c["fallbacks"]) == (st["duplicates"], st["visible"], st["fallbacks"])
    assert got.shape == want.shape
    if fmt == "f32":
        d = (got - want).abs().max().item()
        assert d <= 1e-4, d
    assert torch.equal(got, want)


def test_two_calls_in_a_row_the_second_smaller(ctx):
    big = synth.c2_scene(1_000_000).subset(np.arange(0, 1_000_000, 6))  # 166,667 Gaussians
    s1 = ctx.load_scene(big)
    traj = synth.c2_trajectory(41)
    _say("call 1: 166,667 Gaussians (1M/720p scene subset), 1280x720, pose 40")
    _same(ctx, s1, traj[40], synth.fov_intrinsics(1280, 720), 1280, 720, "f32")
    c1s, c1p, c1k, c1w, c1h = synth.c1_single_view()
    s2 = ctx.load_scene(c1s)
    _say("call 2: 20k Gaussians, 256x256")
    _same(ctx, s2, c1p[0], c1k, c1w, c1h, "f32")
    _say("call 3: 20k Gaussians, 256x256 RGB8 at rung 0.5, SH degree 1")
    _same(ctx, s2, c1p[0], c1k, c1w, c1h, "rgb8", res_scale=0.5, sh_degree=1)
    s1.free()
    s2.free()


def test_overflowing_call_gives_background_then_next_call_is_exact(ctx):
    sc = synth.scene_uniform(seed=5, n=20000)
    sc.log_scales[:] = 0.5  # every Gaussian covers much of a 1080p frame: far more pairs than the array holds
    sc.opacity_logits[:] = 4.0
    s = ctx.load_scene(sc)
    pose = synth.Pose(np.eye(3, dtype=np.float32), np.array([0.0, 0.0, -3.0], np.float32))
    k = synth.fov_intrinsics(1920, 1080)
    _say("overflow: 20k Gaussians of scale e^0.5 at 1920x1080")
    got, c = _noalloc(ctx, s, pose, k, 1920, 1080, "f32", bg=(0.25, 0.5, 0.75))
    _say("counters", c)
    assert c["overflow"] == 1
    bg = torch.tensor([0.25, 0.5, 0.75], device="cuda").expand_as(got)
    assert torch.equal(got, bg)
    s.free()
    c1s, c1p, c1k, c1w, c1h = synth.c1_single_view()
    s2 = ctx.load_scene(c1s)
    _say("after the overflow: 20k Gaussians, 256x256")
    _same(ctx, s2, c1p[0], c1k, c1w, c1h, "f32")
    s2.free()


def test_scene_too_large_for_the_array_is_refused(ctx):
    sc = synth.scene_uniform(seed=6, n=800_000)
    s = ctx.load_scene(sc)
    out = torch.empty((256, 256, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(tigas.TigasError) as e:
        ctx.render_noalloc(s, synth.Pose(np.eye(3, dtype=np.float32), np.array([0, 0, -3], np.float32)),
                           synth.fov_intrinsics(256, 256), 256, 256, out)
    assert e.value.status == -1 and "scratch" in str(e.value)
    s.free()


def test_host_frame_is_refused(ctx):
    c1s, c1p, c1k, c1w, c1h = synth.c1_single_view()
    s = ctx.load_scene(c1s)
    out = torch.empty((c1h, c1w, 3), dtype=torch.uint8)
    with pytest.raises(tigas.TigasError) as e:
        ctx.render_noalloc(s, c1p[0], c1k, c1w, c1h, out)
    assert e.value.status == -1
    s.free()
