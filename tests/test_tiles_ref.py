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
