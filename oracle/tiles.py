"""CPU reference of the duplicate / sort / tile-range stage (test infrastructure only).

Given per-Gaussian screen footprints (inclusive pixel bounding boxes), tile
counts and FP32 depth-key bits, this rebuilds the duplicate list the way the
method defines it -- one entry per (Gaussian, overlapped tile), key =
(tile id << 32) | depth bits, value = Gaussian index, emitted in Gaussian
order and row-major over each Gaussian's tile rectangle -- orders it with
numpy's stable argsort (a library routine) and derives each tile's
[start, end) range.  Used to check the GPU's keys, values and ranges
byte for byte.  tile_keep adds the tighter tile culling the GPU can apply to
the same entries (the Gaussian must reach the skip threshold somewhere in the
tile), computed from the GPU's own per-Gaussian exponent coefficients.
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


def entries(rects, counts):
    """(Gaussian, tx, ty) of every entry in emission order: Gaussians in index
    order, each one's tiles row-major over its rectangle."""
    counts = np.asarray(counts, np.int64)
    total = int(counts.sum())
    if total == 0:
        z = np.zeros(0, np.int64)
        return z, z, z
    g = np.repeat(np.arange(counts.shape[0], dtype=np.int64), counts)
    start = np.cumsum(counts) - counts
    local = np.arange(total, dtype=np.int64) - start[g]
    nx = (rects[:, 2] - rects[:, 0] + 1)[g]
    tx = rects[g, 0] + local % nx
    ty = rects[g, 1] + local // nx
    return g, tx, ty


def duplicates(rects, counts, zbits, tiles_x: int, keep=None):
    """Keys (uint64) and values (uint32) in emission order; with `keep` (one
    flag per entry of the full rectangles, as tile_keep returns) only the
    kept entries."""
    g, tx, ty = entries(rects, counts)
    if g.size == 0:
        return np.zeros(0, np.uint64), np.zeros(0, np.uint32)
    if keep is not None:
        g, tx, ty = g[keep], tx[keep], ty[keep]
    tile = (ty * tiles_x + tx).astype(np.uint64)
    keys = (tile << np.uint64(32)) | np.asarray(zbits, np.uint64)[g]
    return keys, g.astype(np.uint32)


F = np.float32
LOG2_ALPHA_MIN = F(-7.99435343685886)  # log2(1/255) as the FP32 constant both sides use


def tile_keep(rec, rects, counts, width: int, height: int, tile_w: int, tile_h: int):
    """Tighter tile culling: for every entry of the full rectangles (emission
    order), whether the Gaussian's exponent e(d) = A dx^2 + B dx dy + C dy^2 + L
    (log2 units) can reach the skip threshold log2(1/255) somewhere on the
    rectangle of the tile's pixel centres inside the frame.  The maximum of
    the concave quadratic over a rectangle is at its centre when the centre
    lies inside, else on a face facing the centre, where it is a concave
    function of one variable maximised at its clamped stationary point; the
    threshold is lowered by a rounding margin (0.02 plus 1e-5 (|A|+|B|+|C|) r^2)
    so that only tiles whose every pixel skips the Gaussian are dropped.
    Evaluated in FP32, one rounding per operation in the order written, no
    fused operations: the decisions the GPU's test takes.  rec: per Gaussian
    (u_hi, v_hi, u_lo, v_lo, A, B, C, L, ...) as the preprocess wrote them."""
    g, tx, ty = entries(rects, counts)
    r = np.asarray(rec, F)[g]
    uhi, vhi, ulo, vlo, A, B, C, L = (r[:, k] for k in range(8))
    ox = (tx * tile_w).astype(F)
    oy = (ty * tile_h).astype(F)
    cw = np.minimum(tile_w, width - tx * tile_w).astype(F)
    ch = np.minimum(tile_h, height - ty * tile_h).astype(F)
    with np.errstate(all="ignore"):
        u = (uhi - ox) + ulo
        v = (vhi - oy) + vlo
        dx0 = F(0.5) - u
        dx1 = (cw - F(0.5)) - u
        dy0 = F(0.5) - v
        dy1 = (ch - F(0.5)) - v
        concave = (A < 0) & (C < 0) & (B * B < (F(4.0) * A) * C)
        inside = (dx0 <= 0) & (dx1 >= 0) & (dy0 <= 0) & (dy1 >= 0)
        cx = np.where(dx1 < 0, dx1, dx0)
        sy = np.fmin(np.fmax((-B * cx) / (F(2.0) * C), dy0), dy1)
        ex = (A * cx + B * sy) * cx + (C * sy) * sy
        cy = np.where(dy1 < 0, dy1, dy0)
        sx = np.fmin(np.fmax((-B * cy) / (F(2.0) * A), dx0), dx1)
        ey = (C * cy + B * sx) * cy + (A * sx) * sx
        q = np.where(inside, F(0.0), np.fmax(ex, ey))
        r2 = np.fmax(dx0 * dx0, dx1 * dx1) + np.fmax(dy0 * dy0, dy1 * dy1)
        margin = F(0.02) + (F(1e-5) * ((np.abs(A) + np.abs(B)) + np.abs(C))) * r2
        below = q + L < LOG2_ALPHA_MIN - margin
    return ~concave | ~below


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
