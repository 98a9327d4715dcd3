"""Python front end of the JPEG oracle (test infrastructure only).

Only the tests and the benchmark's CPU-baseline leg import this module; the
product path never does.  The encoder lives in ``jpeg.c`` (plain C, the
steps of a baseline JPEG written out from the standard); this file builds it
with gcc when it is missing and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jpeg.c")
_LIB_PATH = os.path.join(_HERE, "libjpegoracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile jpeg.c into libjpegoracle.so with gcc."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        _lib.orc_jpeg.restype = ctypes.c_int64
        _lib.orc_jpeg.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.c_int64]
        _lib.orc_jpeg_coeffs.restype = None
        _lib.orc_jpeg_coeffs.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        _lib.orc_jpeg_qtable.restype = None
        _lib.orc_jpeg_qtable.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        _lib.orc_jpeg_htable.restype = ctypes.c_int
        _lib.orc_jpeg_htable.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    return _lib


def _rgb(img):
    a = np.ascontiguousarray(img, dtype=np.uint8)
    assert a.ndim == 3 and a.shape[2] == 3
    return a


def encode(img, quality: int) -> bytes:
    """Baseline JPEG of an H x W x 3 uint8 image."""
    a = _rgb(img)
    H, W = a.shape[:2]
    cap = 4096 + 3 * 2 * W * H
    out = np.zeros(cap, np.uint8)
    n = lib().orc_jpeg(a.ctypes.data, W, H, int(quality), out.ctypes.data, cap)
    assert n <= cap
    return out[:n].tobytes()


def coeffs(img, quality: int) -> np.ndarray:
    """Quantised coefficients [blocks, 8, 8] (MCU order: Y, Cb, Cr per MCU)."""
    a = _rgb(img)
    H, W = a.shape[:2]
    nb = ((W + 7) // 8) * ((H + 7) // 8) * 3
    out = np.zeros((nb, 64), np.int32)
    lib().orc_jpeg_coeffs(a.ctypes.data, W, H, int(quality), out.ctypes.data)
    return out.reshape(nb, 8, 8)


def qtable(quality: int, chroma: bool) -> np.ndarray:
    out = np.zeros(64, np.uint8)
    lib().orc_jpeg_qtable(int(quality), int(chroma), out.ctypes.data)
    return out.reshape(8, 8)


def htable(t: int):
    """(code counts per length 1..16, symbols) of table t: 0 DC luma, 1 AC luma,
    2 DC chroma, 3 AC chroma."""
    n = np.zeros(16, np.uint8)
    s = np.zeros(162, np.uint8)
    m = lib().orc_jpeg_htable(int(t), n.ctypes.data, s.ctypes.data)
    return n, s[:m]
