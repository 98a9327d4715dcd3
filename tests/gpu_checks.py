"""Comparisons of the HIP path's outputs with the FP64 oracle (used by the GPU tests)."""
import math

import numpy as np

from oracle import oracle as orc
from oracle import tiles as tref

LOG2E = 1.4426950408889634
TOL_FRAME = 1e-4   # max |delta| per channel for FP32 frames


def k1_fields(dbg):
    r = dbg["rec"].astype(np.float64)
    return dict(u=r[:, 0] + r[:, 2], v=r[:, 1] + r[:, 3],
                con_a=r[:, 4] / (-0.5 * LOG2E), con_b=r[:, 5] / (-LOG2E), con_c=r[:, 6] / (-0.5 * LOG2E),
                L=r[:, 7], rgb=r[:, 8:11], opacity=r[:, 11])


def support_pixels(proj, W, H):
    """Inclusive pixel ranges whose centres lie in the FP64 support box."""
    u, v = proj.field("u"), proj.field("v")
    ex, ey = proj.field("ext_x"), proj.field("ext_y")
    x0 = np.maximum(np.ceil(u - ex - 0.5), 0)
    x1 = np.minimum(np.floor(u + ex - 0.5), W - 1)
    y0 = np.maximum(np.ceil(v - ey - 0.5), 0)
    y1 = np.minimum(np.floor(v + ey - 0.5), H - 1)
    has = proj.valid & (ex > 0) & (x0 <= x1) & (y0 <= y1)
    return np.stack([x0, y0, x1, y1], 1).astype(np.int64), has


KAPPA = 64.0       # FP64 conic fallback when a*c > KAPPA * det


def fallback_sets(proj, margin=1.01):
    """Gaussians whose FP64 condition number a*c/det is clearly above (sure to
    take the FP64 fallback) or clearly below (sure not to) the threshold; the
    GPU decides in FP32, so a thin band around it is left out of both."""
    a, c, det = proj.field("a"), proj.field("c"), proj.field("det")
    with np.errstate(divide="ignore", invalid="ignore"):
        kappa = np.where(det > 0, a * c / det, np.inf)
    return kappa > KAPPA * margin, kappa < KAPPA / margin


def check_preprocess(dbg, proj, W, H):
    """K1 against the FP64 per-Gaussian values; returns a dict of worst errors.
    Conic tolerance: 1e-4 relative for ordinary Gaussians, 1e-6 for those
    inverted on the FP64 path."""
    f = k1_fields(dbg)
    touched = dbg["touched"] > 0
    # identical FP32 depth keys everywhere both sides define them
    np.testing.assert_array_equal(dbg["zkey"], proj.zkey)
    # every Gaussian with a support pixel in the image is visible on the GPU,
    # and its GPU pixel box contains those pixels
    box, has = support_pixels(proj, W, H)
    assert np.all(touched[has]), "a Gaussian with oracle support in the image was dropped"
    gb = dbg["bbox"]
    inside = (gb[has, 0] <= box[has, 0]) & (gb[has, 1] <= box[has, 1]) & \
             (gb[has, 2] >= box[has, 2]) & (gb[has, 3] >= box[has, 3])
    assert np.all(inside), "GPU footprint does not cover the oracle support"
    # GPU-visible Gaussians are valid for the oracle
    assert np.all(proj.valid[touched])
    m = touched
    err = {}
    err["uv"] = float(max(np.abs(f["u"][m] - proj.field("u")[m]).max(initial=0),
                          np.abs(f["v"][m] - proj.field("v")[m]).max(initial=0)))
    scale = np.abs(proj.field("con_a")) + np.abs(proj.field("con_c"))
    cerr = np.max(np.stack([np.abs(f[k] - proj.field(k)) for k in ("con_a", "con_b", "con_c")]), axis=0)
    rel = np.where(m, cerr / np.where(scale > 0, scale, 1.0), 0.0)
    sure_fb, sure_plain = fallback_sets(proj)
    err["conic_rel"] = float(rel[m & ~sure_fb].max(initial=0))
    err["conic_rel_fp64"] = float(rel[m & sure_fb].max(initial=0))
    err["n_fp64"] = int(np.sum(m & sure_fb))
    orgb = np.stack([proj.field("r"), proj.field("g"), proj.field("b_")], 1)
    err["rgb"] = float(np.abs(f["rgb"][m] - orgb[m]).max(initial=0))
    err["opacity_rel"] = float((np.abs(f["opacity"][m] - proj.field("opacity")[m]) /
                                proj.field("opacity")[m]).max(initial=0))
    assert err["uv"] <= 1e-3, err
    assert err["conic_rel"] <= 1e-4, err
    assert err["conic_rel_fp64"] <= 1e-6, err
    assert err["rgb"] <= 1e-5, err
    assert err["opacity_rel"] <= 1e-6, err
    return err


def check_tiles(dbg, tile_w, tile_h, cull=False):
    """Keys, values and ranges byte-identical to the CPU reference built from
    the GPU's own per-Gaussian footprints and depth keys (with cull, less the
    entries the tile test drops, decided from the GPU's own exponent
    coefficients)."""
    bbox = dbg["bbox"].astype(np.int64)
    rects, counts = tref.tile_rects(bbox, tile_w, tile_h)
    np.testing.assert_array_equal(counts, dbg["touched"].astype(np.int64))
    keep = None
    if cull:
        H, W = dbg["image"].shape[:2]
        keep = tref.tile_keep(dbg["rec"], rects, counts, W, H, tile_w, tile_h)
    keys, vals = tref.duplicates(rects, counts, dbg["zkey"], dbg["tiles_x"], keep=keep)
    assert keys.shape[0] == dbg["n_dup"]
    # the GPU emits Gaussians in depth order (its depth digits are sorted first)
    ek, ev = tref.depth_first_emission(keys, vals)
    np.testing.assert_array_equal(dbg["keys"], ek)
    np.testing.assert_array_equal(dbg["vals"], ev)
    sk, sv, rg = tref.sort_and_ranges(keys, vals, dbg["tiles_x"] * dbg["tiles_y"])
    np.testing.assert_array_equal(dbg["skeys"], sk)
    np.testing.assert_array_equal(dbg["svals"], sv)
    np.testing.assert_array_equal(dbg["ranges"], rg)


def check_frame_pixels(gpu_rgb, branches, nb, tol=TOL_FRAME):
    """n_bad: pixels matching none of their oracle branches within tol
    (unresolved pixels included, compared with the branches the oracle did
    follow); n_unresolved: pixels whose decision forks exceeded the oracle's
    budget.  A parity test asserts both are zero."""
    best, ok = orc.match(gpu_rgb, branches, nb, tol)
    unresolved = int(np.sum(nb.reshape(-1) < 0))
    bad = np.nonzero(~ok)[0]
    return dict(max_dist=float(best[np.isfinite(best)].max(initial=0)), n_bad=int(bad.size),
                n_unresolved=unresolved, n=int(best.size), bad_idx=bad[:10])


def psnr(a, b):
    a = np.clip(np.asarray(a, np.float64), 0, 1)
    b = np.clip(np.asarray(b, np.float64), 0, 1)
    mse = np.mean((a - b) ** 2)
    return math.inf if mse == 0 else 10 * math.log10(1.0 / mse)


def round_attrs(scene, storage):
    """The scene as the library stores it: attributes rounded to FP16 / BF16
    (nearest even), centres kept in FP32."""
    from paper_2605_08699_amd.synth import Scene

    def bf16(a):
        u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
        return (u.astype(np.uint32) << 16).view(np.float32)

    r = (lambda a: np.asarray(a, np.float32).astype(np.float16).astype(np.float32)) if storage == "f16" else bf16
    return Scene(scene.means.copy(), r(scene.log_scales), r(scene.quats), r(scene.opacity_logits), r(scene.sh),
                 scene.sh_degree)
