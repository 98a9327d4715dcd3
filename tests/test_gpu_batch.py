"""Batched form (needs an MI355X): many views of uneven resolution in one
launch sequence with a persistent blend, replayed from captured HIP graphs,
tile shape and batch depth chosen by the autotuner.  Every frame must be
bit-identical to rendering the view alone, and the views of the 32-view
batch match the FP64 oracle on sampled pixels."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2605_08699_amd import synth, tigas
from tests import gpu_checks as gc
from tests.handmade import random_tiny_scene

pytestmark = pytest.mark.gpu

RUNGS = synth.RUNG_SCALES


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = tigas.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c2small():
    scene = synth.c2_scene(200_000)
    traj = synth.c2_trajectory(64)
    return scene, traj, synth.fov_intrinsics(1280, 720)


@pytest.mark.parametrize("tile,ppl", [((16, 16), 1), ((8, 8), 1), ((16, 32), 1), ((16, 16), 2), ((32, 16), 2)])
def test_batch_equals_single_renders(ctx, c2small, tile, ppl):
    scene, traj, k = c2small
    s = ctx.load_scene(scene)
    poses = [traj[i] for i in range(0, 64, 8)]
    scales = [RUNGS[i % 4] for i in range(len(poses))]
    ks = [k] * len(poses)
    got = ctx.render_batch([s] * len(poses), poses, ks, [1280] * len(poses), [720] * len(poses), scales,
                           fmt="f32", tile=tile, batch_depth=64, ppl=ppl)
    for i, p in enumerate(poses):
        want = ctx.render(s, p, k, 1280, 720, res_scale=scales[i], fmt="f32", tile=(8, 8), batch_depth=64)
        np.testing.assert_array_equal(got[i], want, err_msg=f"view {i} rung {scales[i]}")
    st = ctx.stats()
    _say("batch", tile, st)
    s.free()


@pytest.mark.parametrize("tile", [(16, 16), (16, 32)])
def test_culled_batch_equals_whole_rectangle_batch(ctx, c2small, tile):
    """A batch of uneven views (global tile ids over several grids) with the
    tighter tile culling: the same frames, fewer entries."""
    scene, traj, k = c2small
    s = ctx.load_scene(scene)
    poses = [traj[i] for i in range(0, 64, 8)]
    scales = [RUNGS[i % 4] for i in range(len(poses))]
    ks = [k] * len(poses)
    args = ([s] * len(poses), poses, ks, [1280] * len(poses), [720] * len(poses), scales)
    full = ctx.render_batch(*args, fmt="f32", tile=tile, batch_depth=64)
    d_full = ctx.stats()["duplicates"]
    ctx.set_tile_culling(True)
    try:
        got = ctx.render_batch(*args, fmt="f32", tile=tile, batch_depth=64)
        d_culled = ctx.stats()["duplicates"]
    finally:
        ctx.set_tile_culling(False)
    _say("culled batch", tile, d_culled, "of", d_full)
    for i in range(len(poses)):
        np.testing.assert_array_equal(got[i], full[i], err_msg=f"view {i}")
    assert d_culled < d_full
    s.free()


def test_batch_of_several_scenes_and_rgb8(ctx, c2small):
    scene, traj, k = c2small
    other = random_tiny_scene(np.random.default_rng(5), n=5000, extent=2.0, depth=(3.0, 8.0))
    sa = ctx.load_scene(scene)
    sb = ctx.load_scene(other, "f16")
    scenes = [sa, sa, sb, sa, sb, sb]
    poses = [traj[0], traj[10], synth.Pose(np.eye(3, dtype=np.float32), np.zeros(3, np.float32)), traj[20],
             synth.Pose(np.eye(3, dtype=np.float32), np.array([0.1, 0, 0], np.float32)),
             synth.Pose(np.eye(3, dtype=np.float32), np.array([0, 0.1, 0], np.float32))]
    scales = [1.0, 0.5, 0.75, 0.25, 1.0, 0.5]
    got = ctx.render_batch(scenes, poses, [k] * 6, [1280] * 6, [720] * 6, scales, fmt="rgb8", tile=(16, 16),
                           batch_depth=128)
    for i in range(6):
        want = ctx.render(scenes[i], poses[i], k, 1280, 720, res_scale=scales[i], fmt="rgb8", tile=(16, 16),
                          batch_depth=128)
        np.testing.assert_array_equal(got[i], want, err_msg=f"view {i}")
    sa.free()
    sb.free()


def test_graph_replays_match_eager(ctx, c2small):
    # replay the captured step several times with eager work and syncs in
    # between; every replay must equal the eager (uncaptured) result
    scene, traj, k = c2small
    s = ctx.load_scene(scene)
    poses = [traj[i] for i in range(0, 32, 4)]
    scales = [RUNGS[i % 4] for i in range(len(poses))]
    n = len(poses)
    ctx.set_graphs(False)
    eager = ctx.render_batch([s] * n, poses, [k] * n, [1280] * n, [720] * n, scales, fmt="f32", tile=(16, 16),
                             batch_depth=64)
    ctx.set_graphs(True)
    for rep in range(4):
        got = ctx.render_batch([s] * n, poses, [k] * n, [1280] * n, [720] * n, scales, fmt="f32", tile=(16, 16),
                               batch_depth=64)
        for i in range(n):
            np.testing.assert_array_equal(got[i], eager[i], err_msg=f"replay {rep} view {i}")
        # eager work and a different shape in between
        ctx.set_graphs(False)
        ctx.render(s, traj[40 + rep], k, 1280, 720, fmt="f32", tile=(8, 8), batch_depth=64)
        ctx.set_graphs(True)
    # single-view graphs replay too, with new poses each time
    ctx.set_graphs(False)
    ref = [ctx.render(s, traj[i], k, 1280, 720, fmt="f32", tile=(16, 16), batch_depth=64) for i in range(5)]
    ctx.set_graphs(True)
    for rep in range(2):
        for i in range(5):
            got = ctx.render(s, traj[i], k, 1280, 720, fmt="f32", tile=(16, 16), batch_depth=64)
            np.testing.assert_array_equal(got, ref[i], err_msg=f"single replay {rep} pose {i}")
    s.free()


def test_autotuner_choice_does_not_change_frames(ctx, c2small):
    scene, traj, k = c2small
    s = ctx.load_scene(scene)
    poses = [traj[i] for i in range(0, 40, 5)]
    scales = [RUNGS[i % 4] for i in range(len(poses))]
    n = len(poses)
    auto = ctx.render_batch([s] * n, poses, [k] * n, [1280] * n, [720] * n, scales, fmt="f32")
    st = ctx.stats()
    _say("autotuned", st["tile_w"], st["tile_h"], st["batch_depth"], st["pixels_per_lane"])
    assert (st["tile_w"], st["tile_h"]) in [(8, 8), (16, 16), (16, 32), (32, 16)]  # the candidate shapes
    assert st["batch_depth"] in (64, 128, 256) and st["pixels_per_lane"] in (1, 2)
    fixed = ctx.render_batch([s] * n, poses, [k] * n, [1280] * n, [720] * n, scales, fmt="f32", tile=(16, 16),
                             batch_depth=64)
    for i in range(n):
        np.testing.assert_array_equal(auto[i], fixed[i])
    s.free()


def test_batched_3m_scene_32_views_match_single_renders_and_oracle(ctx):
    # the 32-view batch of the 3M-Gaussian scene at four rungs: every view
    # equals its single render bit for bit, and sampled pixels of every view
    # match the FP64 oracle within 1e-4
    scene = synth.c3_scene()
    poses, scales = synth.c4_views()
    k = synth.fov_intrinsics(1920, 1080)
    s = ctx.load_scene(scene)
    n = len(poses)
    got = ctx.render_batch([s] * n, poses, [k] * n, [1920] * n, [1080] * n, scales, fmt="f32", tile=(16, 32),
                           batch_depth=64)
    st = ctx.stats()
    _say("32 views", st)
    assert st["tiles"] == 8 * sum(-(-round(1920 * r) // 16) * -(-round(1080 * r) // 32) for r in RUNGS)
    rng = np.random.default_rng(4)
    for i in range(n):
        want = ctx.render(s, poses[i], k, 1920, 1080, res_scale=scales[i], fmt="f32", tile=(16, 16),
                          batch_depth=64)
        np.testing.assert_array_equal(got[i], want, err_msg=f"view {i}")
        proj = orc.preprocess(scene, poses[i], k, 1920, 1080, scale=scales[i])
        idx = rng.choice(proj.out_w * proj.out_h, 150, replace=False)
        px, py = idx % proj.out_w, idx // proj.out_w
        br, nb = orc.render_pixels(proj, px, py)
        res = gc.check_frame_pixels(got[i][py, px], br, nb)
        assert res["n_bad"] == 0 and res["n_unresolved"] == 0, (i, res)
    s.free()


def test_scene_reloaded_after_free_renders_its_own_data(ctx, c2small):
    # captured graphs hold a scene's device pointers: a scene loaded after
    # another was freed (possibly at the same host address) must never replay
    # the freed scene's graph
    scene, traj, k = c2small
    other = synth.scene_clusters(seed=77, n=scene.n, n_clusters=16, surface_frac=0.2)
    fresh = tigas.Context(0)
    try:
        for rep in range(3):
            sa = ctx.load_scene(scene)
            a = ctx.render(sa, traj[1], k, 1280, 720, fmt="f32", tile=(16, 16), batch_depth=64)
            sa.free()
            sb = ctx.load_scene(other)
            b = ctx.render(sb, traj[1], k, 1280, 720, fmt="f32", tile=(16, 16), batch_depth=64)
            sb.free()
            fb = fresh.load_scene(other)
            want = fresh.render(fb, traj[1], k, 1280, 720, fmt="f32", tile=(16, 16), batch_depth=64)
            fb.free()
            np.testing.assert_array_equal(b, want, err_msg=f"reload {rep}")
            assert not np.array_equal(a, b)
    finally:
        fresh.close()
