"""Pins of the JPEG oracle (CPU): tables against libjpeg's (through Pillow),
decodability and quality of its streams with an independent decoder, and
closed forms of the transform.  The ladder's quality factors come from the
paper's Table 1 (10, 35, 65, 90)."""
import io
import math

import numpy as np
import pytest
from PIL import Image

from oracle import jpeg as oj

LADDER_Q = (10, 35, 65, 90)


def _test_image(H, W, seed=0):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:H, 0:W]
    img = np.stack([128 + 100 * np.sin(x / 7.0 + y / 11.0), 128 + 90 * np.cos(y / 5.0),
                    (x * 3 + y * 2) % 256], -1)
    img = img + rng.normal(0, 6, img.shape)
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def _decode(b):
    return np.asarray(Image.open(io.BytesIO(b)).convert("RGB"))


def _psnr(a, b):
    mse = ((a.astype(np.float64) - b.astype(np.float64)) ** 2).mean()
    return 10 * math.log10(255.0 ** 2 / max(mse, 1e-12))


def _libjpeg(img, q):
    buf = io.BytesIO()
    Image.fromarray(img).save(buf, "JPEG", quality=q, subsampling=0)
    return buf.getvalue()


def _segments(b):
    """(marker, payload) of the header segments up to SOS."""
    out, i = [], 2
    while i < len(b):
        assert b[i] == 0xFF
        m = b[i + 1]
        n = (b[i + 2] << 8) | b[i + 3]
        out.append((m, b[i + 4:i + 2 + n]))
        i += 2 + n
        if m == 0xDA:
            break
    return out, i


@pytest.mark.parametrize("q", [1, 10, 35, 50, 65, 90, 100])
def test_quantisation_tables_match_libjpeg(q):
    im = Image.open(io.BytesIO(_libjpeg(_test_image(16, 16), q)))
    ref = im.quantization
    np.testing.assert_array_equal(oj.qtable(q, False).reshape(-1), np.array(ref[0], np.uint8))
    np.testing.assert_array_equal(oj.qtable(q, True).reshape(-1), np.array(ref[1], np.uint8))


def test_huffman_tables_match_libjpeg():
    segs, _ = _segments(_libjpeg(_test_image(16, 16), 75))
    tables = {}
    for m, p in segs:
        if m != 0xC4:
            continue
        i = 0
        while i < len(p):
            tc_th = p[i]
            counts = np.frombuffer(p[i + 1:i + 17], np.uint8)
            n = int(counts.sum())
            tables[tc_th] = (counts, np.frombuffer(p[i + 17:i + 17 + n], np.uint8))
            i += 17 + n
    for t, key in ((0, 0x00), (1, 0x10), (2, 0x01), (3, 0x11)):
        counts, syms = oj.htable(t)
        np.testing.assert_array_equal(counts, tables[key][0])
        np.testing.assert_array_equal(syms, tables[key][1])


@pytest.mark.parametrize("size", [(1, 1), (8, 8), (9, 17), (37, 53), (64, 96)])
def test_streams_decode_and_quality_rises_with_q(size):
    H, W = size
    img = _test_image(H, W, seed=H * 100 + W)
    sizes, psnrs = [], []
    for q in LADDER_Q + (100,):
        b = oj.encode(img, q)
        d = _decode(b)
        assert d.shape == img.shape
        sizes.append(len(b))
        psnrs.append(_psnr(d, img))
    assert sizes == sorted(sizes)
    assert psnrs[-1] > 40.0 and psnrs[3] > 30.0
    if H * W >= 64 * 64:
        assert psnrs == sorted(psnrs)


@pytest.mark.parametrize("q", LADDER_Q)
def test_decoded_image_close_to_libjpeg_at_the_same_quality(q):
    img = _test_image(72, 120, seed=q)
    a = _decode(oj.encode(img, q))
    b = _decode(_libjpeg(img, q))
    # two encoders of the same standard with the same tables: they differ only
    # in the rounding of the transform
    assert _psnr(a, b) > 36.0
    assert abs(_psnr(a, img) - _psnr(b, img)) < 1.0


def test_constant_image_has_dc_only():
    img = np.empty((16, 24, 3), np.uint8)
    img[...] = (200, 100, 50)
    c = oj.coeffs(img, 100)  # unit quantiser steps
    assert np.count_nonzero(c[:, 1:, :]) == 0 and np.count_nonzero(c[:, 0, 1:]) == 0
    y = 0.299 * 200 + 0.587 * 100 + 0.114 * 50
    cb = -0.168736 * 200 - 0.331264 * 100 + 0.5 * 50
    cr = 0.5 * 200 - 0.418688 * 100 - 0.081312 * 50
    # orthonormal DCT: the DC coefficient is 8 x the block mean
    for comp, v in enumerate((y - 128.0, cb, cr)):
        assert np.all(np.abs(c[comp::3, 0, 0] - 8.0 * v) <= 0.5 + 1e-3)
    d = _decode(oj.encode(img, 90)).astype(int)
    assert np.abs(d - img.astype(int)).max() <= 2


@pytest.mark.parametrize("freq", [1, 3, 6])
@pytest.mark.parametrize("vertical", [False, True])
def test_cosine_pattern_gives_one_coefficient(freq, vertical):
    # f = 128 + A cos((2n+1) u pi / 16) along one axis: F(0, u) (or F(u, 0)) =
    # 4 sqrt(2) A, every other coefficient zero up to the 8-bit rounding of f
    A = 100.0
    n = np.arange(8)
    wave = 128 + A * np.cos((2 * n + 1) * freq * np.pi / 16)
    g = np.tile(wave, (8, 1)) if not vertical else np.tile(wave[:, None], (1, 8))
    img = np.repeat(np.clip(np.rint(g), 0, 255).astype(np.uint8)[..., None], 3, axis=2)
    c = oj.coeffs(img, 100)[0].astype(float)  # the Y block
    k, l = (freq, 0) if vertical else (0, freq)
    assert abs(c[k, l] - 4 * math.sqrt(2) * A) <= 3.0
    rest = c.copy()
    rest[k, l] = 0
    assert np.abs(rest).max() <= 3.0


def test_restart_markers_and_byte_stuffing():
    img = _test_image(40, 64, seed=5)  # 40 MCUs: no restart marker
    assert oj.encode(img, 90).count(b"\xff\xd0") == 0
    img = _test_image(40, 136, seed=5)
    img[:8] = 255  # saturated rows push 0xFF bytes into the entropy-coded data
    b = oj.encode(img, 100)
    _, i = _segments(b)
    data = b[i:-2]
    assert b[-2:] == b"\xff\xd9"
    rst, j = [], 0
    while j < len(data):
        if data[j] == 0xFF:
            nxt = data[j + 1]
            assert nxt == 0x00 or 0xD0 <= nxt <= 0xD7
            if nxt != 0x00:
                rst.append(nxt - 0xD0)
            j += 2
        else:
            j += 1
    n_mcu = ((40 + 7) // 8) * ((136 + 7) // 8)
    assert rst == [r % 8 for r in range((n_mcu + 39) // 40 - 1)]  # intervals of 40 MCUs
    assert data.count(b"\xff\x00") > 0
    assert _psnr(_decode(b), img) > 40.0
