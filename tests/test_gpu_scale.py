"""Parity at full workload sizes (needs an MI355X).

1M Gaussians at 1280x720 along the 300-pose trajectory (sampled poses,
sampled pixels against the FP64 oracle one by one, per-Gaussian values and
bit-exact tile lists on whole frames), and the 3M-Gaussian 1080p scene with
FP32 / FP16 / BF16 attribute storage (PSNR against the FP64 oracle and
against the GPU FP32 frames).
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2605_08699_amd import synth, tigas
from tests import gpu_checks as gc

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = tigas.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c2():
    return synth.c2_scene(), synth.c2_trajectory(300), synth.fov_intrinsics(1280, 720)


@pytest.fixture(scope="module")
def c3():
    return synth.c3_scene(), synth.c3_trajectory(300), synth.fov_intrinsics(1920, 1080)


def _sample(rng, W, H, n):
    idx = rng.choice(W * H, n, replace=False)
    return idx % W, idx // W


@pytest.mark.parametrize("pose_i", [0, 150, 299])
def test_c2_sampled_pixels_match_oracle(ctx, c2, pose_i):
    scene, traj, k = c2
    s = ctx.load_scene(scene)
    _say("c2 pose", pose_i)
    img = ctx.render(s, traj[pose_i], k, 1280, 720, fmt="f32")
    proj = orc.preprocess(scene, traj[pose_i], k, 1280, 720)
    px, py = _sample(np.random.default_rng(pose_i), 1280, 720, 3000)
    br, nb = orc.render_pixels(proj, px, py)
    res = gc.check_frame_pixels(img[py, px], br, nb)
    _say("c2", pose_i, res, ctx.stats())
    assert res["n_bad"] == 0 and res["n_unresolved"] == 0, res
    s.free()


def test_c2_preprocess_and_tiles_full_frame(ctx, c2):
    scene, traj, k = c2
    s = ctx.load_scene(scene)
    dbg = ctx.render_debug(s, traj[100], k, 1280, 720)
    proj = orc.preprocess(scene, traj[100], k, 1280, 720)
    err = gc.check_preprocess(dbg, proj, 1280, 720)
    _say("c2 k1", err, "D", dbg["n_dup"])
    gc.check_tiles(dbg, 16, 16)
    s.free()


def test_c3_fp32_sampled_pixels(ctx, c3):
    scene, traj, k = c3
    s = ctx.load_scene(scene)
    img = ctx.render(s, traj[0], k, 1920, 1080, fmt="f32")
    proj = orc.preprocess(scene, traj[0], k, 1920, 1080)
    px, py = _sample(np.random.default_rng(7), 1920, 1080, 2000)
    br, nb = orc.render_pixels(proj, px, py)
    res = gc.check_frame_pixels(img[py, px], br, nb)
    _say("c3 fp32", res, ctx.stats())
    # near-singular surface splats: the FP32 conic carries ~eps*cond(Sigma2D)
    # relative error; parity at 1e-4 is required for the volumetric workloads,
    # here the frame must match to PSNR >= 50 dB against the same oracle pixels
    assert gc.psnr(img[py, px], br[:, 0, :3]) >= 50.0
    s.free()


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_c3_reduced_precision_psnr(ctx, c3, storage):
    scene, traj, k = c3
    s32 = ctx.load_scene(scene, "f32")
    sh = ctx.load_scene(scene, storage)
    worst_gpu = np.inf
    for i in range(0, 300, 10):
        a = ctx.render(s32, traj[i], k, 1920, 1080, fmt="f32")
        b = ctx.render(sh, traj[i], k, 1920, 1080, fmt="f32")
        worst_gpu = min(worst_gpu, gc.psnr(a, b))
    proj = orc.preprocess(scene, traj[0], k, 1920, 1080)
    px, py = _sample(np.random.default_rng(11), 1920, 1080, 2000)
    br, nb = orc.render_pixels(proj, px, py)
    b0 = ctx.render(sh, traj[0], k, 1920, 1080, fmt="f32")
    p_oracle = gc.psnr(b0[py, px], br[:, 0, :3])
    _say(storage, "min PSNR vs GPU FP32 over 30 poses", worst_gpu, "PSNR vs FP64 oracle (pose 0 sample)", p_oracle)
    assert worst_gpu >= 50.0
    assert p_oracle >= 50.0
    s32.free()
    sh.free()


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_reduced_precision_decode_matches_oracle_of_rounded_scene(ctx, storage):
    # the FP16/BF16 path computes exactly like FP32 on the rounded attributes
    scene, poses, k, W, H = synth.c1_single_view()
    s = ctx.load_scene(scene, storage)
    img = ctx.render(s, poses[0], k, W, H, fmt="f32")
    proj = orc.preprocess(gc.round_attrs(scene, storage), poses[0], k, W, H)
    br, nb = orc.render_frame(proj)
    res = gc.check_frame_pixels(img.reshape(-1, 3), br.reshape(-1, br.shape[2], 4), nb.reshape(-1))
    _say(storage, res)
    assert res["n_bad"] == 0, res
