"""CPU reference of the duplicate / sort / tile-range stage (test infrastructure only).

Given per-Gaussian screen footprints (inclusive pixel bounding boxes), tile
counts and FP32 depth-key bits, this rebuilds the duplicate list the way the
method defines it -- one entry per (Gaussian, overlapped tile), key =
(tile id << 32) | depth bits, value = Gaussian index, emitted in Gaussian
order and row-major over each Gaussian's tile rectangle -- orders it with
numpy's stable argsort (a library routine) and derives each tile's
[start, end) range.  Used to check the GPU's keys, values and ranges
byte for byte.
"""
from __future__ import annotations

import numpy as np


def tile_rects(bbox, tile_w: int, tile_h: int):
    """Tile rectangles [tx0, ty0, tx1, ty1] (inclusive) of inclusive pixel boxes
    [x0, y0, x1, y1]; empty boxes (x1 < x0 or y1 < y0) give zero tiles."""
    b = np.asarray(bbox, np.int64).reshape(-1, 4)
    empty = (b[:, 2] < b[:, 0]) | (b[:, 3] < b[:, 1])
    tx0 = b[:, 0] // tile_w
    ty0 = b[:, 1] // tile_h
    tx1 = b[:, 2] // tile_w
    ty1 = b[:, 3] // tile_h
    count = (tx1 - tx0 + 1) * (ty1 - ty0 + 1)
    count[empty] = 0
    return np.stack([tx0, ty0, tx1, ty1], 1), count


def duplicates(rects, counts, zbits, tiles_x: int):
    """Keys (uint64) and values (uint32) in emission order."""
    counts = np.asarray(counts, np.int64)
    total = int(counts.sum())
    if total == 0:
        return np.zeros(0, np.uint64), np.zeros(0, np.uint32)
    g = np.repeat(np.arange(counts.shape[0], dtype=np.int64), counts)
    start = np.cumsum(counts) - counts
    local = np.arange(total, dtype=np.int64) - start[g]
    nx = (rects[:, 2] - rects[:, 0] + 1)[g]
    tx = rects[g, 0] + local % nx
    ty = rects[g, 1] + local // nx
    tile = (ty * tiles_x + tx).astype(np.uint64)
    keys = (tile << np.uint64(32)) | np.asarray(zbits, np.uint64)[g]
    return keys, g.astype(np.uint32)


def sort_and_ranges(keys, vals, n_tiles: int):
    """Stable sort by key; per-tile [start, end) ranges of the sorted list
    ((0, 0) for a tile without entries)."""
    order = np.argsort(keys, kind="stable")
    sk = keys[order]
    sv = vals[order]
    tiles = (sk >> np.uint64(32)).astype(np.int64)
    t = np.arange(n_tiles + 1, dtype=np.int64)
    bounds = np.searchsorted(tiles, t, side="left")
    ranges = np.stack([bounds[:-1], bounds[1:]], 1).astype(np.uint32)
    ranges[ranges[:, 0] == ranges[:, 1]] = 0
    return sk, sv, ranges


def depth_first_emission(keys, vals):
    """The duplicate list in the order a depth-first emitter produces it:
    Gaussians taken in (depth, index) order, each with its tiles row-major.
    That is the record-order list stably sorted by the depth word alone."""
    order = np.argsort(keys & np.uint64(0xFFFFFFFF), kind="stable")
    return keys[order], vals[order]
