"""Python front end of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module; the product path never does.  The arithmetic lives in
``oracle.c`` (plain C, FP64, OpenMP over pixels); this file marshals numpy
arrays, builds the C library with gcc when it is missing, and holds the
set-valued comparison used by the parity tests.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

NF = 16
FIELDS = ("u", "v", "z", "a", "b", "c", "con_a", "con_b", "con_c", "opacity",
          "r", "g", "b_", "ext_x", "ext_y", "det")
F = {name: i for i, name in enumerate(FIELDS)}

# relative widths of the decision bands inside which the oracle follows both
# outcomes of a threshold test (alpha vs 1/255, T' vs 1e-4)
BAND_ALPHA = 1e-4
BAND_T = 1e-3
MAX_BRANCHES = 4


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        L.orc_rung.argtypes = [D, D, D, D, ctypes.c_int, ctypes.c_int, D, P, P, P]
        L.orc_rung.restype = None
        L.orc_sh_basis_many.argtypes = [I64, P, P]
        L.orc_sh_basis_many.restype = None
        L.orc_sh_color.argtypes = [ctypes.c_int, P, P, P]
        L.orc_sh_color.restype = None
        L.orc_preprocess.argtypes = [I64, P, P, P, P, P, ctypes.c_int, P, P, P, P, P, P]
        L.orc_preprocess.restype = I64
        L.orc_depth_order.argtypes = [I64, P, P, P]
        L.orc_depth_order.restype = I64
        L.orc_prefilter_boxes.argtypes = [I64, P, D, P]
        L.orc_prefilter_boxes.restype = None
        L.orc_render_pixels.argtypes = [I64, P, P, I64, P, P, P, D, D, ctypes.c_int, P, P]
        L.orc_render_pixels.restype = None
        L.orc_pack_rgb8.argtypes = [I64, P, P]
        L.orc_pack_rgb8.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    lib().orc_set_threads(int(n))


def rung(intr, width: int, height: int, scale: float = 1.0):
    """(out_w, out_h, (fx, fy, cx, cy)) of a resolution-scaled render."""
    ow = ctypes.c_int()
    oh = ctypes.c_int()
    k = np.zeros(4, np.float64)
    lib().orc_rung(float(intr.fx), float(intr.fy), float(intr.cx), float(intr.cy), int(width), int(height),
                   float(np.float32(scale)), ctypes.byref(ow), ctypes.byref(oh), _p(k))
    return ow.value, oh.value, tuple(float(x) for x in k)


def sh_basis(dirs) -> np.ndarray:
    """Real SH basis (16 functions, degree <= 3) at unit directions [K,3]."""
    d = np.ascontiguousarray(np.asarray(dirs, np.float64).reshape(-1, 3))
    Y = np.zeros((d.shape[0], 16), np.float64)
    lib().orc_sh_basis_many(d.shape[0], _p(d), _p(Y))
    return Y


def sh_color(deg: int, direction, coeffs) -> np.ndarray:
    d = np.ascontiguousarray(np.asarray(direction, np.float64).reshape(3))
    k = np.ascontiguousarray(np.asarray(coeffs, np.float64).reshape(48))
    out = np.zeros(3, np.float64)
    lib().orc_sh_color(int(deg), _p(d), _p(k), _p(out))
    return out


class Projected:
    """Per-Gaussian FP64 values of one view."""

    def __init__(self, values, zkey, valid, out_w, out_h, cam):
        self.values = values          # [N, NF] float64
        self.zkey = zkey              # [N] uint32 FP32 order-key bits
        self.valid = valid            # [N] bool
        self.out_w = out_w
        self.out_h = out_h
        self.cam = cam                # (fx, fy, cx, cy) of the output image
        self._order = None
        self._sorted = None
        self._boxes = None

    def field(self, name):
        return self.values[:, F[name]]

    @property
    def order(self) -> np.ndarray:
        if self._order is None:
            n = self.zkey.shape[0]
            order = np.zeros(max(n, 1), np.int64)
            valid8 = np.ascontiguousarray(self.valid.astype(np.uint8))
            m = lib().orc_depth_order(n, _p(self.zkey), _p(valid8), _p(order))
            self._order = order[:m].copy()
        return self._order

    def sorted_values(self) -> np.ndarray:
        if self._sorted is None:
            self._sorted = np.ascontiguousarray(self.values[self.order])
        return self._sorted

    def boxes(self, band_a=BAND_ALPHA) -> np.ndarray:
        if self._boxes is None:
            sv = self.sorted_values()
            b = np.zeros((max(sv.shape[0], 1), 4), np.float64)
            lib().orc_prefilter_boxes(sv.shape[0], _p(sv), float(band_a), _p(b))
            self._boxes = b
        return self._boxes


def preprocess(scene, pose, intr, width: int, height: int, scale: float = 1.0, sh_degree=None) -> Projected:
    """FP64 per-Gaussian projection of ``scene`` for one camera."""
    L = lib()
    n = scene.n
    deg = scene.sh_degree if sh_degree is None else int(sh_degree)
    ow, oh, k4 = rung(intr, width, height, scale)
    cam = np.array([k4[0], k4[1], k4[2], k4[3], ow, oh], np.float64)
    f32 = lambda a: np.ascontiguousarray(np.asarray(a, np.float32))
    means, ls, q, op, sh = (f32(scene.means), f32(scene.log_scales), f32(scene.quats),
                            f32(scene.opacity_logits), f32(scene.sh))
    R = f32(pose.R).reshape(9)
    t = f32(pose.t).reshape(3)
    vals = np.zeros((max(n, 1), NF), np.float64)
    zkey = np.zeros(max(n, 1), np.uint32)
    valid = np.zeros(max(n, 1), np.uint8)
    L.orc_preprocess(n, _p(means), _p(ls), _p(q), _p(op), _p(sh), deg, _p(R), _p(t), _p(cam),
                     _p(vals), _p(zkey), _p(valid))
    return Projected(vals[:n], zkey[:n], valid[:n].astype(bool), ow, oh, k4)


def render_pixels(proj: Projected, px, py, bg=(0.0, 0.0, 0.0), prefilter: bool = True,
                  band_a: float = BAND_ALPHA, band_t: float = BAND_T, max_branches: int = MAX_BRANCHES):
    """Set-valued FP64 colours of the pixels (px[i], py[i]).

    Returns (branches [npix, max_branches, 4] = (r, g, b, T_final), nbranch [npix]);
    nbranch < 0 marks a pixel whose decision forks exceeded the budget."""
    px = np.ascontiguousarray(np.asarray(px, np.int32).reshape(-1))
    py = np.ascontiguousarray(np.asarray(py, np.int32).reshape(-1))
    sv = proj.sorted_values()
    box = proj.boxes(band_a) if prefilter else None
    bgv = np.asarray(bg, np.float64).reshape(3).copy()
    out = np.zeros((px.shape[0], max_branches, 4), np.float64)
    nb = np.zeros(px.shape[0], np.int32)
    lib().orc_render_pixels(sv.shape[0], _p(sv), _p(box) if box is not None else None, px.shape[0],
                            _p(px), _p(py), _p(bgv), float(band_a), float(band_t), int(max_branches),
                            _p(out), _p(nb))
    return out, nb


def render_frame(proj: Projected, bg=(0.0, 0.0, 0.0), **kw):
    """All pixels of the output image; branches reshaped to [H, W, B, 4]."""
    H, W = proj.out_h, proj.out_w
    yy, xx = np.mgrid[0:H, 0:W]
    out, nb = render_pixels(proj, xx.reshape(-1), yy.reshape(-1), bg, **kw)
    return out.reshape(H, W, -1, 4), nb.reshape(H, W)


def render_nominal(proj: Projected, bg=(0.0, 0.0, 0.0), prefilter: bool = True) -> np.ndarray:
    """Single-valued FP64 frame [H, W, 3] (no decision forks)."""
    out, nb = render_frame(proj, bg, prefilter=prefilter, band_a=0.0, band_t=0.0, max_branches=1)
    return out[:, :, 0, :3]


def pack_rgb8(frame) -> np.ndarray:
    """8-bit frame of an FP32 frame [..., 3]: round half up of 255 * clamp(c, 0, 1) in FP32."""
    f = np.ascontiguousarray(np.asarray(frame, np.float32))
    out = np.zeros(f.shape, np.uint8)
    lib().orc_pack_rgb8(f.size, _p(f), _p(out))
    return out


def match(gpu_rgb, branches, nbranch, tol: float):
    """Per pixel: the max-abs distance of the GPU colour to the closest oracle
    branch, and whether it is within ``tol``.  gpu_rgb: [..., 3]."""
    g = np.asarray(gpu_rgb, np.float64).reshape(-1, 1, 3)
    br = branches.reshape(g.shape[0], -1, 4)[:, :, :3]
    nb = np.abs(np.asarray(nbranch).reshape(-1))
    dist = np.max(np.abs(br - g), axis=2)
    mask = np.arange(br.shape[1])[None, :] < nb[:, None]
    dist = np.where(mask, dist, np.inf)
    best = dist.min(axis=1)
    return best, best <= tol
