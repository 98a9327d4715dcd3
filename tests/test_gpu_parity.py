"""Parity of the HIP path with the FP64 oracle (needs an MI355X).

Every call goes through the C ABI of libtigas.so via the ctypes binding.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2605_08699_amd import synth, tigas
from tests import gpu_checks as gc
from tests.handmade import eye_pose, intr, make_scene, random_tiny_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tigas.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c1():
    return synth.c1_single_view()


def _say(*a):
    print(*a, flush=True)


def test_wave_scan_dpp():
    rng = np.random.default_rng(0)
    for n in (64, 200, 4096 + 17):
        x = rng.integers(0, 1000, n).astype(np.uint32)
        got = tigas.selftest_wave_scan(x)
        want = np.concatenate([np.cumsum(x[i:i + 64]) for i in range(0, n, 64)]).astype(np.uint32)
        np.testing.assert_array_equal(got, want)


def test_c1_preprocess_matches_oracle(ctx, c1):
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    _say("c1 preprocess", scene.n, W, H)
    dbg = ctx.render_debug(s, poses[0], k, W, H)
    proj = orc.preprocess(scene, poses[0], k, W, H)
    err = gc.check_preprocess(dbg, proj, W, H)
    _say("k1 errors", err)
    assert err["uv"] < 1e-4


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 32), (32, 16)])
def test_c1_tile_lists_sort_and_ranges_bit_exact(ctx, c1, tile):
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    _say("c1 tiles", tile)
    dbg = ctx.render_debug(s, poses[0], k, W, H, tile=tile)
    gc.check_tiles(dbg, *tile)
    assert dbg["n_dup"] > scene.n


def test_c1_frame_matches_oracle(ctx, c1):
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    img = ctx.render(s, poses[0], k, W, H, fmt="f32")
    proj = orc.preprocess(scene, poses[0], k, W, H)
    br, nb = orc.render_frame(proj)
    res = gc.check_frame_pixels(img.reshape(-1, 3), br.reshape(-1, br.shape[2], 4), nb.reshape(-1))
    _say("c1 frame", res)
    assert res["n_bad"] == 0 and res["n_unresolved"] == 0, res
    st = ctx.stats()
    _say("stats", st)
    assert st["visible"] > 0 and st["duplicates"] > 0


def test_c1_rgb8_is_the_packed_f32_frame(ctx, c1):
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    f = ctx.render(s, poses[0], k, W, H, fmt="f32", bg=(0.2, 0.3, 0.4))
    b = ctx.render(s, poses[0], k, W, H, fmt="rgb8", bg=(0.2, 0.3, 0.4))
    want = np.floor(np.clip(f, 0, 1).astype(np.float32) * np.float32(255) + np.float32(0.5)).astype(np.uint8)
    np.testing.assert_array_equal(b, want)


def test_frames_bit_identical_across_tiles_and_batch_depths(ctx, c1):
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    ref = ctx.render(s, poses[0], k, W, H, fmt="f32")
    for tile in [(8, 8), (16, 16), (16, 32), (32, 16)]:
        for bd in (64, 128, 256):
            for ppl in ((1,) if tile[1] < 16 else (1, 2)):
                got = ctx.render(s, poses[0], k, W, H, fmt="f32", tile=tile, batch_depth=bd, ppl=ppl)
                np.testing.assert_array_equal(got, ref, err_msg=f"tile={tile} bd={bd} ppl={ppl}")


def test_render_is_deterministic(ctx, c1):
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    a = ctx.render(s, poses[0], k, W, H, fmt="f32")
    b = ctx.render(s, poses[0], k, W, H, fmt="f32")
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("size", [(1, 1), (7, 13), (33, 17), (100, 1)])
def test_ragged_and_tiny_images(ctx, size):
    W, H = size
    rng = np.random.default_rng(W * 100 + H)
    scene = random_tiny_scene(rng, n=300, extent=1.0)
    k = intr(max(W, H) * 0.9, W / 2, H / 2)
    s = ctx.load_scene(scene)
    _say("ragged", size)
    for tile in [(16, 16), (8, 8)]:
        dbg = ctx.render_debug(s, eye_pose(), k, W, H, tile=tile)
        gc.check_tiles(dbg, *tile)
        proj = orc.preprocess(scene, eye_pose(), k, W, H)
        gc.check_preprocess(dbg, proj, W, H)
        br, nb = orc.render_frame(proj)
        res = gc.check_frame_pixels(dbg["image"].reshape(-1, 3), br.reshape(-1, br.shape[2], 4), nb.reshape(-1))
        assert res["n_bad"] == 0, res


@pytest.mark.parametrize("size", [(2048, 24), (2072, 24), (24, 2072)])
def test_wide_views_both_rectangle_encodings(ctx, size):
    # up to 256 x 256 tiles a view's tile rectangles travel packed in one word
    # through the depth passes; beyond that (here 259 tiles of 8 px) the last
    # depth pass gathers them: lists and pixels must match either way
    W, H = size
    rng = np.random.default_rng(W + 7 * H)
    scene = random_tiny_scene(rng, n=400, extent=1.0)
    axis = 0 if W > H else 1
    scene.means[:, axis] *= 7.0
    k = intr(700.0, W / 2, H / 2)
    s = ctx.load_scene(scene)
    _say("wide", size)
    dbg = ctx.render_debug(s, eye_pose(), k, W, H, tile=(8, 8))
    gc.check_tiles(dbg, 8, 8)
    proj = orc.preprocess(scene, eye_pose(), k, W, H)
    gc.check_preprocess(dbg, proj, W, H)
    br, nb = orc.render_frame(proj)
    res = gc.check_frame_pixels(dbg["image"].reshape(-1, 3), br.reshape(-1, br.shape[2], 4), nb.reshape(-1))
    assert res["n_bad"] == 0, res
    assert dbg["n_dup"] > 0
    if max(W, H) > 2048:  # Gaussians reach the tiles past 255
        assert dbg["bbox"][:, 2 + axis].max() >= 2048


def test_empty_scene_and_all_culled_render_background(ctx):
    bg = (0.25, 0.5, 0.75)
    empty = make_scene(np.zeros((0, 3)))
    s = ctx.load_scene(empty)
    img = ctx.render(s, eye_pose(), intr(50, 20, 20), 40, 40, fmt="f32", bg=bg)
    np.testing.assert_array_equal(img, np.broadcast_to(np.float32(bg), img.shape))
    behind = make_scene([[0, 0, -3], [0, 0, 0.1], [50, 0, 3]], log_scales=[[math.log(0.3)] * 3] * 3)
    s2 = ctx.load_scene(behind)
    img = ctx.render(s2, eye_pose(), intr(50, 20, 20), 40, 40, fmt="f32", bg=bg)
    np.testing.assert_array_equal(img, np.broadcast_to(np.float32(bg), img.shape))
    assert ctx.stats()["duplicates"] == 0


def test_nan_and_zero_quaternion_are_dropped(ctx):
    sc = make_scene([[0, 0, 3], [0.1, 0, 3], [0, 0.1, 3], [0, 0, 4], [0.05, 0.05, 3], [-0.1, 0, 3.5],
                     [0, -0.1, 3.5]], log_scales=[[math.log(0.2)] * 3] * 7,
                    logits=[2] * 7, colors=[[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]] + [[0.5, 0.5, 0.5]] * 3,
                    sh_degree=3)
    sc.quats[1] = 0
    sc.means[2, 1] = np.nan
    sc.log_scales[3, 0] = np.inf
    sc.sh[4, 12, 1] = np.nan          # a degree-3 coefficient
    sc.sh[5, 0, 2] = -np.inf          # the DC term
    sc.opacity_logits[6] = np.inf
    s = ctx.load_scene(sc)
    k = intr(60, 16, 16)
    img = ctx.render(s, eye_pose(), k, 32, 32, fmt="f32")
    proj = orc.preprocess(sc, eye_pose(), k, 32, 32)
    np.testing.assert_array_equal(proj.valid, [True, False, False, False, False, False, False])
    assert np.isfinite(img).all()
    br, nb = orc.render_frame(proj)
    res = gc.check_frame_pixels(img.reshape(-1, 3), br.reshape(-1, br.shape[2], 4), nb.reshape(-1))
    assert res["n_bad"] == 0, res


def test_closed_form_saturated_layers(ctx):
    bg = (0.1, 0.2, 0.3)
    c1c = np.array([0.9, 0.8, 0.7])
    sc = make_scene([[0, 0, 2], [0, 0, 3], [0, 0, 4]], log_scales=[[math.log(5.0)] * 3] * 3,
                    logits=[10.0] * 3, colors=[c1c, [0, 1, 0], [1, 0, 0]])
    s = ctx.load_scene(sc)
    img = ctx.render(s, eye_pose(), intr(50, 4, 4), 8, 8, fmt="f32", bg=bg).astype(np.float64)
    col = 0.5 + (0.5 / math.sqrt(math.pi)) * sc.sh[0, 0].astype(np.float64)
    want = float(np.float32(0.99)) * col + (1 - float(np.float32(0.99))) * np.array(bg)
    np.testing.assert_allclose(img, np.broadcast_to(want, img.shape), atol=1e-6)


def test_rungs_and_principal_point(ctx, c1):
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    for sc in (0.25, 0.5, 0.75):
        img = ctx.render(s, poses[0], k, W, H, res_scale=sc, fmt="f32")
        proj = orc.preprocess(scene, poses[0], k, W, H, scale=sc)
        assert img.shape[:2] == (proj.out_h, proj.out_w)
        br, nb = orc.render_frame(proj)
        res = gc.check_frame_pixels(img.reshape(-1, 3), br.reshape(-1, br.shape[2], 4), nb.reshape(-1))
        _say("rung", sc, res)
        assert res["n_bad"] == 0, res


def test_invalid_arguments_are_reported(ctx, c1):
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    with pytest.raises(tigas.TigasError, match="E_INVALID"):
        ctx.render(s, poses[0], k, W, H, tile=(12, 12))
    with pytest.raises(tigas.TigasError, match="E_INVALID"):
        ctx.render(s, poses[0], k, 0, H)
    bad = synth.Pose(np.full((3, 3), np.nan, np.float32), np.zeros(3, np.float32))
    with pytest.raises(tigas.TigasError, match="E_INVALID"):
        ctx.render(s, bad, k, W, H)


def test_single_pass_sort_gives_the_same_lists_and_frames(ctx, c1):
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    big = ctx.load_scene(synth.c2_scene(1_000_000))
    traj = synth.c2_trajectory(8)
    k2 = synth.fov_intrinsics(1280, 720)
    ref = [ctx.render(big, traj[i], k2, 1280, 720, fmt="f32", tile=(16, 16)) for i in range(3)]
    ctx.set_sort(True)
    try:
        _say("single-pass sort")
        for tile in [(16, 16), (8, 8)]:
            dbg = ctx.render_debug(s, poses[0], k, W, H, tile=tile)
            gc.check_tiles(dbg, *tile)
        for rep in range(2):  # captured graphs replay with fresh look-back epochs
            for i in range(3):
                got = ctx.render(big, traj[i], k2, 1280, 720, fmt="f32", tile=(16, 16))
                np.testing.assert_array_equal(got, ref[i], err_msg=f"rep {rep} pose {i}")
        _say("single-pass stats", ctx.stats())
        assert ctx.sort_fallbacks() == 0
    finally:
        ctx.set_sort(False)
        big.free()


def test_kernel_timing_brackets_every_launch(ctx, c1):
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    ref = ctx.render(s, poses[0], k, W, H, fmt="f32")
    ctx.profile_kernels(True)
    try:
        for _ in range(3):
            got = ctx.render(s, poses[0], k, W, H, fmt="f32")
        kt = ctx.kernel_times()
    finally:
        ctx.profile_kernels(False)
    _say("kernel times", kt)
    np.testing.assert_array_equal(got, ref)
    pre = [n for n in kt if "k_preprocess<0, 3>" in n]
    blend = [n for n in kt if "k_blend<" in n]
    assert len(pre) == 1 and kt[pre[0]][0] == 3
    assert len(blend) == 1 and kt[blend[0]][0] == 3
    assert all(ms > 0 for _, ms in kt.values())


def test_block_culling_never_changes_a_pixel(ctx, monkeypatch):
    # the blend drops, per wave, entries whose exponent stays below the skip
    # threshold on its whole block; frames must equal those rendered without it
    scene = synth.c3_scene()
    traj = synth.c3_trajectory(300)
    k = synth.fov_intrinsics(1920, 1080)
    monkeypatch.setenv("TIGAS_BLEND_CULL", "0")
    plain = tigas.Context(0)
    monkeypatch.delenv("TIGAS_BLEND_CULL")
    try:
        sa = ctx.load_scene(scene)
        sb = plain.load_scene(scene)
        for i in (0, 75, 150, 225):
            for tile, ppl in (((16, 32), 1), ((16, 16), 2), ((8, 8), 1)):
                _say("cull check pose", i, tile, ppl)
                a = ctx.render(sa, traj[i], k, 1920, 1080, fmt="f32", tile=tile, batch_depth=64, ppl=ppl)
                b = plain.render(sb, traj[i], k, 1920, 1080, fmt="f32", tile=tile, batch_depth=64, ppl=ppl)
                np.testing.assert_array_equal(a, b, err_msg=f"pose {i} tile {tile} ppl {ppl}")
        ea, ca = ctx.count_blend_work(sa, traj[0], k, 1920, 1080, tile=(16, 32), batch_depth=64, ppl=1)
        eb, cb = plain.count_blend_work(sb, traj[0], k, 1920, 1080, tile=(16, 32), batch_depth=64, ppl=1)
        _say("evaluations with / without culling", ea, eb, "contributions", ca, cb)
        assert ca == cb and ea <= eb
        sa.free()
        sb.free()
    finally:
        plain.close()
