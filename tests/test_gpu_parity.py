"""Parity of the HIP path with the FP64 oracle (needs an MI355X).

Every call goes through the C ABI of libtigas.so via the ctypes binding.
"""
import ctypes
import dataclasses
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


@pytest.mark.parametrize("binning", [True, False])
@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 32), (32, 16)])
def test_c1_tile_lists_sort_and_ranges_bit_exact(ctx, c1, tile, binning):
    """Both placements of the tile digit (counting, radix passes) give the
    sorted list of the plain 64-bit key sort."""
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    _say("c1 tiles", tile, "binning", binning)
    ctx.set_tile_binning(binning)
    try:
        dbg = ctx.render_debug(s, poses[0], k, W, H, tile=tile)
        passes = ctx.stats()["sort_passes"]
    finally:
        ctx.set_tile_binning(True)
    gc.check_tiles(dbg, *tile)
    assert dbg["n_dup"] > scene.n
    # 3 depth passes, then one counting placement or the radix tile passes
    assert passes == (4 if binning else 3 + math.ceil(math.log2((W // tile[0]) * (H // tile[1])) / 8))


@pytest.mark.parametrize("binning", [True, False])
def test_c1_three_and_four_pass_depth_sorts_give_identical_lists_and_frames(ctx, c1, binning):
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    got = {}
    ctx.set_tile_binning(binning)
    try:
        for passes in (3, 4):
            ctx.set_depth_passes(passes)
            dbg = ctx.render_debug(s, poses[0], k, W, H, tile=(16, 16))
            got[passes] = (dbg, ctx.stats())
    finally:
        ctx.set_depth_passes(3)
        ctx.set_tile_binning(True)
    _say("depth passes", {p: g[1]["sort_passes"] for p, g in got.items()})
    tile_passes = 1 if binning else math.ceil(math.log2((W // 16) * (H // 16)) / 8)
    for passes, (dbg, st) in got.items():
        gc.check_tiles(dbg, 16, 16)
        assert st["rerenders"] == 0
        assert st["sort_passes"] == passes + tile_passes
    for key in ("svals", "skeys", "ranges", "image"):
        np.testing.assert_array_equal(got[3][0][key], got[4][0][key])


def test_depth_passes_other_than_three_or_four_are_refused(ctx):
    for bad in (0, 2, 5, -1):
        with pytest.raises(tigas.TigasError, match="E_INVALID"):
            ctx.set_depth_passes(bad)
    ctx.set_depth_passes(3)


def test_frame_too_deep_for_three_passes_is_rendered_again_with_four():
    # depths from 0.5 to 2e7 (their FP32 keys span more than 2^27), sizes
    # growing with depth so that every Gaussian covers a few pixels
    rng = np.random.default_rng(5)
    n = 600
    z = np.exp(rng.uniform(math.log(0.5), math.log(2e7), n))
    means = np.column_stack([rng.uniform(-0.35, 0.35, n) * z, rng.uniform(-0.25, 0.25, n) * z, z])
    ls = np.repeat(np.log(0.02 * z)[:, None], 3, axis=1) + rng.normal(0.0, 0.3, (n, 3))
    scene = make_scene(means, ls, rng.normal(size=(n, 4)), rng.normal(1.0, 1.0, n), rng.uniform(0.0, 1.0, (n, 3)))
    W, H = 200, 136
    k = intr(150.0, W / 2, H / 2)
    c = tigas.Context(0)  # the switch to four passes is kept per context
    try:
        s = c.load_scene(scene)
        img = c.render(s, eye_pose(), k, W, H, fmt="f32", tile=(16, 16))
        st = c.stats()
        _say("deep frame", st)
        assert st["rerenders"] == 1 and st["sort_passes"] == 5
        proj = orc.preprocess(scene, eye_pose(), k, W, H)
        br, nb = orc.render_frame(proj)
        res = gc.check_frame_pixels(img.reshape(-1, 3), br.reshape(-1, br.shape[2], 4), nb.reshape(-1))
        assert res["n_bad"] == 0 and res["n_unresolved"] == 0, res
        # later frames take four passes from the start
        dbg = c.render_debug(s, eye_pose(), k, W, H, tile=(16, 16))
        st2 = c.stats()
        assert st2["rerenders"] == 0 and st2["sort_passes"] == 5
        zk = dbg["zkey"][dbg["touched"] > 0].astype(np.int64)
        assert zk.max() - (zk.min() & ~511) >= 1 << 27  # the frame is too deep for three passes
        gc.check_tiles(dbg, 16, 16)
        np.testing.assert_array_equal(img, dbg["image"])
    finally:
        c.close()


def test_frame_just_shallow_enough_keeps_three_passes(ctx):
    # the same construction with depths from 0.5 to 1000: keys span less than 2^27
    rng = np.random.default_rng(6)
    n = 600
    z = np.exp(rng.uniform(math.log(0.5), math.log(1000.0), n))
    means = np.column_stack([rng.uniform(-0.35, 0.35, n) * z, rng.uniform(-0.25, 0.25, n) * z, z])
    ls = np.repeat(np.log(0.02 * z)[:, None], 3, axis=1)
    scene = make_scene(means, ls, None, np.full(n, 1.0), rng.uniform(0.0, 1.0, (n, 3)))
    W, H = 200, 136
    k = intr(150.0, W / 2, H / 2)
    s = ctx.load_scene(scene)
    dbg = ctx.render_debug(s, eye_pose(), k, W, H, tile=(16, 16))
    st = ctx.stats()
    zk = dbg["zkey"][dbg["touched"] > 0].astype(np.int64)
    assert 1 << 25 < zk.max() - (zk.min() & ~511) < 1 << 27
    assert st["rerenders"] == 0 and st["sort_passes"] == 4
    gc.check_tiles(dbg, 16, 16)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 32), (32, 16)])
def test_culled_tile_lists_bit_exact_and_frames_unchanged(ctx, c1, tile):
    """Tighter tile culling: the lists equal the reference less exactly the
    entries its tile test drops, fewer entries are sorted, and the frame is
    bit-identical to the one rendered from whole rectangles."""
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    ctx.set_tile_culling(True)
    try:
        dbg = ctx.render_debug(s, poses[0], k, W, H, tile=tile)
        culled = ctx.render(s, poses[0], k, W, H, fmt="f32", tile=tile)
        d_culled = ctx.stats()["duplicates"]
    finally:
        ctx.set_tile_culling(False)
    gc.check_tiles(dbg, *tile, cull=True)
    full = ctx.render(s, poses[0], k, W, H, fmt="f32", tile=tile)
    d_full = ctx.stats()["duplicates"]
    _say("culled", tile, d_culled, "of", d_full)
    np.testing.assert_array_equal(culled, full)
    assert d_culled == dbg["n_dup"] and d_culled < d_full


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
    # the 8-bit frame is the oracle's pack of the FP32 frame, bit for bit ...
    np.testing.assert_array_equal(b, orc.pack_rgb8(f))
    # ... and within one level of the pack of the FP64 oracle's own frame
    proj = orc.preprocess(scene, poses[0], k, W, H)
    nominal = orc.render_nominal(proj, bg=(0.2, 0.3, 0.4)).astype(np.float32)
    assert np.abs(b.astype(int) - orc.pack_rgb8(nominal).astype(int)).max() <= 1


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
        assert res["n_bad"] == 0 and res["n_unresolved"] == 0, res


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
    assert res["n_bad"] == 0 and res["n_unresolved"] == 0, res
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
    assert res["n_bad"] == 0 and res["n_unresolved"] == 0, res


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
        assert res["n_bad"] == 0 and res["n_unresolved"] == 0, res


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
    # an SH degree above the scene's is refused, not clamped
    with pytest.raises(tigas.TigasError, match="E_INVALID"):
        ctx.render(s, poses[0], k, W, H, sh_degree=4)
    s1 = ctx.load_scene(dataclasses.replace(scene, sh_degree=1))
    with pytest.raises(tigas.TigasError, match="E_INVALID"):
        ctx.render(s1, poses[0], k, W, H, sh_degree=2)
    s1.free()


@pytest.mark.parametrize("fmt,scale", [("rgb8", 1.0), ("f32", 0.5)])
def test_small_output_buffer_reports_the_frame_size(ctx, c1, fmt, scale):
    # E_BUFFER for a frame buffer below out_w * out_h * 3 * (1 or 4) bytes;
    # out_w and out_h are written all the same
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    ow, oh = tigas.output_size(W, H, scale)
    need = ow * oh * 3 * (4 if fmt == "f32" else 1)
    buf = np.zeros(need - 1, np.uint8)
    q = tigas.quality_c(scale, -1, fmt)
    fr = tigas.FrameC(ctypes.c_void_p(buf.ctypes.data), buf.nbytes, 0, 0, 0)
    L = tigas.lib()
    rc = L.tigas_render(s.handle, ctypes.byref(tigas.pose_c(poses[0])), ctypes.byref(tigas.intr_c(k)), W, H,
                        ctypes.byref(q), ctypes.byref(fr), None)
    assert rc == -4, rc
    assert (fr.out_w, fr.out_h) == (ow, oh)
    assert "too small" in L.tigas_last_error().decode()
    assert not buf.any()        # nothing was written
    s.free()


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_scenes_of_lower_sh_degree_match_oracle(ctx, c1, deg):
    # a degree-d scene stores only its (d+1)^2 coefficients
    scene, poses, k, W, H = c1
    sc = dataclasses.replace(scene, sh_degree=deg)
    s = ctx.load_scene(sc)
    img = ctx.render(s, poses[0], k, W, H, fmt="f32")
    proj = orc.preprocess(sc, poses[0], k, W, H)
    br, nb = orc.render_frame(proj)
    res = gc.check_frame_pixels(img.reshape(-1, 3), br.reshape(-1, br.shape[2], 4), nb.reshape(-1))
    _say("scene degree", deg, res)
    assert res["n_bad"] == 0 and res["n_unresolved"] == 0, res
    s.free()


@pytest.mark.parametrize("req", [0, 1, 2, 3])
def test_request_sh_degree_at_or_below_the_scenes_matches_oracle(ctx, c1, req):
    scene, poses, k, W, H = c1
    s = ctx.load_scene(scene)
    img = ctx.render(s, poses[0], k, W, H, fmt="f32", sh_degree=req)
    proj = orc.preprocess(scene, poses[0], k, W, H, sh_degree=req)
    br, nb = orc.render_frame(proj)
    res = gc.check_frame_pixels(img.reshape(-1, 3), br.reshape(-1, br.shape[2], 4), nb.reshape(-1))
    _say("request degree", req, res)
    assert res["n_bad"] == 0 and res["n_unresolved"] == 0, res
    s.free()


def _needle_scene(n=40, seed=41):
    """Long thin splats lying in planes facing the camera, their long axis at
    angles across the image plane: seen that way their 2D covariance is close
    to singular (a*c/det far above 64) unless the axis is nearly horizontal or
    vertical."""
    rng = np.random.default_rng(seed)
    means = np.column_stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n), rng.uniform(2.5, 4.0, n)])
    ls = np.column_stack([np.log(rng.uniform(0.08, 0.4, n)), np.log(rng.uniform(1e-4, 3e-3, n)),
                          np.log(rng.uniform(1e-4, 3e-3, n))])
    ang = rng.uniform(0.0, math.pi, n)
    tilt = rng.normal(0.0, 0.05, (n, 2))
    q = np.column_stack([np.cos(ang / 2), tilt[:, 0], tilt[:, 1], np.sin(ang / 2)])
    cols = rng.uniform(0.0, 1.0, (n, 3))
    return make_scene(means, ls, q, rng.normal(1.0, 1.0, n), cols, sh_degree=0)


def test_fp64_fallback_conics_and_pixels_match_oracle(ctx):
    sc = _needle_scene()
    k = intr(220.0, 64, 64)
    s = ctx.load_scene(sc)
    dbg = ctx.render_debug(s, eye_pose(), k, 128, 128)
    st = ctx.stats()
    proj = orc.preprocess(sc, eye_pose(), k, 128, 128)
    sure_fb, _ = gc.fallback_sets(proj)
    vis = dbg["touched"] > 0
    err = gc.check_preprocess(dbg, proj, 128, 128)      # fallback conics within 1e-6 relative
    _say("fallbacks", st["fallbacks"], "sure", int(sure_fb.sum()), err)
    assert int(np.sum(sure_fb & vis)) >= 10
    assert st["fallbacks"] >= int(np.sum(sure_fb & vis))
    br, nb = orc.render_frame(proj)
    res = gc.check_frame_pixels(dbg["image"].reshape(-1, 3), br.reshape(-1, br.shape[2], 4), nb.reshape(-1))
    _say("needles frame", res)
    assert res["n_bad"] == 0 and res["n_unresolved"] == 0, res
    s.free()


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
