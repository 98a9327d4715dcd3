"""Pins of the CPU duplicate/sort/range reference against a pure-Python loop
over tiny inputs (CPU only)."""
import numpy as np

from oracle import tiles


def _brute(bbox, zbits, tw, th, tiles_x, n_tiles):
    entries = []
    for g, (x0, y0, x1, y1) in enumerate(bbox):
        if x1 < x0 or y1 < y0:
            continue
        for ty in range(y0 // th, y1 // th + 1):
            for tx in range(x0 // tw, x1 // tw + 1):
                entries.append(((ty * tiles_x + tx) << 32 | int(zbits[g]), g))
    emitted = list(entries)
    # Python's sort is stable: equal keys keep emission order
    srt = sorted(emitted, key=lambda e: e[0])
    ranges = []
    for t in range(n_tiles):
        idx = [i for i, e in enumerate(srt) if (e[0] >> 32) == t]
        ranges.append((idx[0], idx[-1] + 1) if idx else None)
    return emitted, srt, ranges


def test_reference_matches_python_loops():
    rng = np.random.default_rng(0)
    for trial in range(20):
        W, H, tw, th = 40, 30, [8, 16, 16][trial % 3], [8, 16, 32][trial % 3]
        tiles_x, tiles_y = -(-W // tw), -(-H // th)
        n = 25
        x0 = rng.integers(0, W, n)
        y0 = rng.integers(0, H, n)
        x1 = np.minimum(x0 + rng.integers(-2, 20, n), W - 1)
        y1 = np.minimum(y0 + rng.integers(-2, 20, n), H - 1)
        bbox = np.stack([x0, y0, x1, y1], 1)
        zbits = rng.integers(0x3e000000, 0x3e000010, n).astype(np.uint32)   # many equal depths
        rects, counts = tiles.tile_rects(bbox, tw, th)
        keys, vals = tiles.duplicates(rects, counts, zbits, tiles_x)
        sk, sv, rg = tiles.sort_and_ranges(keys, vals, tiles_x * tiles_y)
        emitted, srt, ranges = _brute(bbox.tolist(), zbits, tw, th, tiles_x, tiles_x * tiles_y)
        assert [(int(k), int(v)) for k, v in zip(keys, vals)] == emitted
        assert [(int(k), int(v)) for k, v in zip(sk, sv)] == srt
        for t, r in enumerate(ranges):
            if r is None:
                assert rg[t, 0] == rg[t, 1]
            else:
                assert tuple(rg[t]) == r


def test_empty_input():
    rects, counts = tiles.tile_rects(np.zeros((0, 4), np.int64), 16, 16)
    keys, vals = tiles.duplicates(rects, counts, np.zeros(0, np.uint32), 4)
    sk, sv, rg = tiles.sort_and_ranges(keys, vals, 12)
    assert keys.size == 0 and np.all(rg == 0)


def test_depth_digits_first_gives_the_same_sorted_list():
    # LSD radix sorting the (tile | depth) keys: sorting the depth digits on one
    # representative per Gaussian before duplicating gives the identical list
    rng = np.random.default_rng(3)
    for trial in range(30):
        n = 60
        x0 = rng.integers(0, 50, n)
        y0 = rng.integers(0, 40, n)
        bbox = np.stack([x0, y0, x0 + rng.integers(-1, 30, n), y0 + rng.integers(-1, 30, n)], 1)
        zbits = rng.integers(0x3e000000, 0x3e000008, n).astype(np.uint32)
        rects, counts = tiles.tile_rects(bbox, 8, 8)
        keys, vals = tiles.duplicates(rects, counts, zbits, 10)
        ref = tiles.sort_and_ranges(keys, vals, 100)
        # depth-first: stable order of Gaussians by depth, then their tiles
        g_order = np.argsort(zbits, kind="stable")
        k2 = []
        v2 = []
        for g in g_order:
            sel = vals == g
            k2.append(keys[sel])
            v2.append(vals[sel])
        k2 = np.concatenate(k2) if k2 else keys
        v2 = np.concatenate(v2) if v2 else vals
        ek, ev = tiles.depth_first_emission(keys, vals)
        np.testing.assert_array_equal(ek, k2)
        np.testing.assert_array_equal(ev, v2)
        # tile-only stable sort of the depth-first list == full key sort
        o = np.argsort(ek >> np.uint64(32), kind="stable")
        np.testing.assert_array_equal(ek[o], ref[0])
        np.testing.assert_array_equal(ev[o], ref[1])


def _random_records(rng, n, W, H):
    """Per-Gaussian (u_hi, v_hi, u_lo, v_lo, A, B, C, L) in the preprocess's
    form: exponent e(d) = A dx^2 + B dx dy + C dy^2 + L in log2 units, with
    conic = inverse of a dilated 2D covariance and L = log2(opacity)."""
    log2e = 1.4426950408889634
    u = rng.uniform(-0.2 * W, 1.2 * W, n)
    v = rng.uniform(-0.2 * H, 1.2 * H, n)
    ang = rng.uniform(0, np.pi, n)
    s1 = np.exp(rng.uniform(np.log(0.3), np.log(0.4 * W), n))
    s2 = s1 * np.exp(rng.uniform(np.log(0.02), 0, n))
    c, s = np.cos(ang), np.sin(ang)
    a = c * c * s1 * s1 + s * s * s2 * s2 + 0.3
    b = c * s * (s1 * s1 - s2 * s2)
    cc = s * s * s1 * s1 + c * c * s2 * s2 + 0.3
    det = a * cc - b * b
    ca, cb, ccon = cc / det, -b / det, a / det
    o = rng.uniform(1.0 / 255.0, 0.99, n)
    uhi = u.astype(np.float32)
    vhi = v.astype(np.float32)
    rec = np.zeros((n, 12), np.float32)
    rec[:, 0], rec[:, 1] = uhi, vhi
    rec[:, 2] = (u - uhi).astype(np.float32)
    rec[:, 3] = (v - vhi).astype(np.float32)
    rec[:, 4] = -0.5 * log2e * ca
    rec[:, 5] = -log2e * cb
    rec[:, 6] = -0.5 * log2e * ccon
    rec[:, 7] = np.log2(o)
    return rec


def _rect_max(abcl, x0, x1, y0, y1):
    """Maximum of A x^2 + B x y + C y^2 + L over [x0, x1] x [y0, y1] (FP64,
    concave quadratic): the centre when inside, else the best point over the
    four edges, each a 1D concave quadratic maximised at its clamped
    stationary point."""
    A, B, C, L = (float(t) for t in abcl)
    f = lambda x, y: A * x * x + B * x * y + C * y * y + L
    if x0 <= 0 <= x1 and y0 <= 0 <= y1:
        return L
    best = -np.inf
    for x in (x0, x1):
        y = min(max(-B * x / (2 * C), y0), y1)
        best = max(best, f(x, y))
    for y in (y0, y1):
        x = min(max(-B * y / (2 * A), x0), x1)
        best = max(best, f(x, y))
    return best


def test_tile_culling_keeps_every_tile_a_gaussian_reaches():
    """Brute force over every pixel centre in FP64: a tile where the exponent
    reaches log2(1/255) at some pixel (so alpha >= 1/255 there) is always
    kept; a tile whose pixels all stay clearly below it (past the rounding
    margin) is dropped, and on these scenes many tiles are."""
    rng = np.random.default_rng(11)
    thr = float(tiles.LOG2_ALPHA_MIN)
    dropped_total = 0
    for W, H, tw, th in ((50, 37, 8, 8), (64, 40, 16, 16), (70, 70, 16, 32)):
        n = 40
        rec = _random_records(rng, n, W, H)
        bbox = np.tile(np.array([[0, 0, W - 1, H - 1]]), (n, 1))  # every tile of the frame
        rects, counts = tiles.tile_rects(bbox, tw, th)
        keep = tiles.tile_keep(rec, rects, counts, W, H, tw, th)
        g, tx, ty = tiles.entries(rects, counts)
        r = rec.astype(np.float64)
        for k in range(g.size):
            gi = g[k]
            xs = np.arange(tx[k] * tw, min((tx[k] + 1) * tw, W)) + 0.5
            ys = np.arange(ty[k] * th, min((ty[k] + 1) * th, H)) + 0.5
            dx = xs[None, :] - (r[gi, 0] + r[gi, 2])
            dy = ys[:, None] - (r[gi, 1] + r[gi, 3])
            e = r[gi, 4] * dx * dx + r[gi, 5] * dx * dy + r[gi, 6] * dy * dy + r[gi, 7]
            emax = e.max()
            if emax >= thr - 1e-4:
                assert keep[k], (gi, tx[k], ty[k], emax)
            # the exact maximum over the continuous rectangle of pixel centres
            # (the test's bound): the centre if inside, else the best clamped
            # stationary point of each of the four edges
            cmax = _rect_max(r[gi, 4:8], dx[0, 0], dx[0, -1], dy[0, 0], dy[-1, 0])
            assert cmax >= emax - 1e-9
            rr = max(dx[0, 0] ** 2, dx[0, -1] ** 2) + max(dy[0, 0] ** 2, dy[-1, 0] ** 2)
            margin = 0.02 + 1e-5 * (abs(r[gi, 4]) + abs(r[gi, 5]) + abs(r[gi, 6])) * rr
            if cmax < thr - margin - 1e-3:
                assert not keep[k], (gi, tx[k], ty[k], cmax, margin)
            dropped_total += int(not keep[k])
    assert dropped_total > 500


def test_tile_culling_list_is_the_rectangle_list_less_the_dropped_entries():
    rng = np.random.default_rng(12)
    W, H, tw, th = 60, 44, 8, 8
    rec = _random_records(rng, 30, W, H)
    x0 = rng.integers(0, W, 30)
    y0 = rng.integers(0, H, 30)
    bbox = np.stack([x0, y0, np.minimum(x0 + rng.integers(0, 25, 30), W - 1),
                     np.minimum(y0 + rng.integers(0, 25, 30), H - 1)], 1)
    rects, counts = tiles.tile_rects(bbox, tw, th)
    zbits = rng.integers(0x3e000000, 0x3e000010, 30).astype(np.uint32)
    keep = tiles.tile_keep(rec, rects, counts, W, H, tw, th)
    full_k, full_v = tiles.duplicates(rects, counts, zbits, -(-W // tw))
    k, v = tiles.duplicates(rects, counts, zbits, -(-W // tw), keep=keep)
    np.testing.assert_array_equal(k, full_k[keep])
    np.testing.assert_array_equal(v, full_v[keep])
    assert 0 < keep.sum() < keep.size
