"""Parity of the GPU JPEG encoder with the JPEG oracle (needs an MI355X): the
streams must be byte-identical.  Every call goes through the C ABI."""
import io
import math

import numpy as np
import pytest
import torch
from PIL import Image

from oracle import jpeg as oj
from paper_2605_08699_amd import synth, tigas

pytestmark = pytest.mark.gpu

LADDER = ((320, 180, 10), (640, 360, 35), (960, 540, 65), (1280, 720, 90))  # Table 1 rungs


@pytest.fixture(scope="module")
def ctx():
    c = tigas.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)


def _image(H, W, seed):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:H, 0:W]
    img = np.stack([128 + 110 * np.sin(x / 5.0 + y / 9.0), 128 + 100 * np.cos(y / 4.0 - x / 13.0),
                    (x * 5 + y * 3) % 256], -1)
    img = img + rng.normal(0, 10, img.shape)
    img[: max(1, H // 5)] = 255  # saturated rows: 0xFF bytes in the coded data
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def _gpu(img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


@pytest.mark.parametrize("size", [(1, 1), (8, 8), (13, 37), (72, 120), (181, 323)])
@pytest.mark.parametrize("q", [1, 10, 35, 65, 90, 100])
def test_stream_equals_oracle(ctx, size, q):
    H, W = size
    img = _image(H, W, seed=H * 7 + W + q)
    _say("jpeg", size, q)
    got = ctx.jpeg_bytes(_gpu(img), q)
    want = oj.encode(img, q)
    assert len(got) == len(want)
    assert got == want


def test_wide_frames_and_repeated_calls(ctx):
    # wide frames (intervals wrap across MCU rows), then a smaller frame on the
    # same buffers, then the large one again: the interval bit buffers must
    # come back cleared
    for H, W, q in ((24, 4096, 90), (16, 40, 35), (24, 4096, 90), (1, 6000, 100), (300, 9, 65)):
        img = _image(H, W, seed=W + H)
        _say("jpeg", (H, W), q)
        assert ctx.jpeg_bytes(_gpu(img), q) == oj.encode(img, q)


def test_rendered_ladder_frames(ctx):
    # frames the rasterizer renders at the ladder's resolutions, encoded at
    # the ladder's quality factors
    scene, poses, _, _, _ = synth.c1_single_view()
    s = ctx.load_scene(scene)
    for w, h, q in LADDER:
        kk = synth.fov_intrinsics(w, h)
        frame = torch.empty((h, w, 3), dtype=torch.uint8, device="cuda")
        ctx.render(s, poses[0], kk, w, h, out=frame)
        _say("jpeg ladder", (w, h), q)
        got = ctx.jpeg_bytes(frame, q)
        img = frame.cpu().numpy()
        assert got == oj.encode(img, q)
        dec = np.asarray(Image.open(io.BytesIO(got)).convert("RGB")).astype(np.float64)
        mse = ((dec - img) ** 2).mean()
        assert 10 * math.log10(255.0 ** 2 / max(mse, 1e-12)) > {10: 25.0, 35: 30.0, 65: 33.0, 90: 38.0}[q]
    s.free()


def test_small_buffer_reports_the_length(ctx):
    img = _image(40, 64, seed=3)
    t = _gpu(img)
    want = oj.encode(img, 90)
    small = torch.zeros(100, dtype=torch.uint8, device="cuda")
    with pytest.raises(tigas.TigasError) as e:
        ctx.jpeg_encode(t, 90, out=small)
    assert "smaller" in str(e.value)
    assert bytes(small.cpu().numpy()) == want[:100]
    out, n = ctx.jpeg_encode(t, 90)
    assert n == len(want) and bytes(out[:n].cpu().numpy()) == want


def test_invalid_arguments(ctx):
    img = _gpu(_image(8, 8, seed=1))
    for q in (0, 101):
        with pytest.raises(tigas.TigasError):
            ctx.jpeg_encode(img, q)
    wide = _gpu(np.zeros((1, 65536, 3), np.uint8))
    with pytest.raises(tigas.TigasError):
        ctx.jpeg_encode(wide, 90)
