"""3DGS PLY reader written from the file format, in plain numpy: test
infrastructure only (the tests use it to check the library's PLY reader and
scene registry; the product reads PLY files in its own C++).

A model file (Section 5.1, PLY Model and Primitives: each scene is parsed from
PLY into centres, log-scales, quaternions, opacity logits and SH
coefficients; the layout is the one the original 3DGS training code writes)
has an element "vertex" with one record per Gaussian:

    x y z                 centre
    f_dc_0 f_dc_1 f_dc_2  SH coefficient 0 of the R, G, B channels
    f_rest_0 .. f_rest_{K-1}
                          the other coefficients, channel-major: with
                          m = K / 3 per channel, f_rest_{c m + k - 1} is
                          coefficient k (1 <= k <= m) of channel c
    opacity               logit
    scale_0..2            log-scales
    rot_0..3              quaternion (w, x, y, z)

K = 3 ((d + 1)^2 - 1) for SH degree d, so 0, 9, 24, 45 for d = 0..3.  The
reader returns the scene arrays of the rasterizer's input layout: means
[n, 3], log_scales [n, 3], quats [n, 4], opacity_logits [n] and sh [n, 16, 3]
(coefficient-major, zero above degree d), each value rounded to FP32.
"""
from __future__ import annotations

import numpy as np

_TYPES = {"char": "i1", "int8": "i1", "uchar": "u1", "uint8": "u1", "short": "i2", "int16": "i2",
          "ushort": "u2", "uint16": "u2", "int": "i4", "int32": "i4", "uint": "u4", "uint32": "u4",
          "float": "f4", "float32": "f4", "double": "f8", "float64": "f8"}


class PlyError(ValueError):
    pass


def read_header(data: bytes):
    """(format, [(element name, count, [(prop, type, list count type or None)])], body offset)."""
    pos = 0
    lines = []
    while True:
        end = data.find(b"\n", pos)
        if end < 0:
            raise PlyError("header has no end_header")
        line = data[pos:end].decode("ascii").rstrip("\r")
        pos = end + 1
        lines.append(line)
        if line.strip() == "end_header":
            break
    if lines[0] != "ply":
        raise PlyError("not a PLY file")
    fmt, elems = None, []
    for line in lines[1:-1]:
        t = line.split()
        if not t or t[0] in ("comment", "obj_info"):
            continue
        if t[0] == "format":
            fmt = t[1]
        elif t[0] == "element":
            elems.append((t[1], int(t[2]), []))
        elif t[0] == "property":
            if t[1] == "list":
                elems[-1][2].append((t[4], _TYPES[t[3]], _TYPES[t[2]]))
            else:
                elems[-1][2].append((t[2], _TYPES[t[1]], None))
        else:
            raise PlyError("unknown header line " + line)
    if fmt not in ("ascii", "binary_little_endian", "binary_big_endian"):
        raise PlyError("unknown format")
    return fmt, elems, pos


def _vertex_columns(fmt, elems, data, pos):
    """{property: float64 column} of the vertex element."""
    vi = [e[0] for e in elems].index("vertex")
    if fmt == "ascii":
        toks = data[pos:].split()
        k = 0
        for name, count, props in elems[:vi]:
            for _ in range(count):
                for _p, _t, lt in props:
                    if lt is None:
                        k += 1
                    else:
                        k += 1 + int(toks[k])
        name, count, props = elems[vi]
        if any(lt is not None for _p, _t, lt in props):
            raise PlyError("list property in the vertex element")
        np_ = len(props)
        vals = toks[k:k + count * np_]
        if len(vals) < count * np_:
            raise PlyError("file ends before the last vertex")
        arr = np.array([float(v) for v in vals], np.float64).reshape(count, np_)
        return {p[0]: arr[:, j] for j, p in enumerate(props)}
    bo = "<" if fmt == "binary_little_endian" else ">"
    for name, count, props in elems[:vi]:
        if all(lt is None for _p, _t, lt in props):
            pos += count * sum(np.dtype(t).itemsize for _p, t, _lt in props)
            continue
        for _ in range(count):
            for _p, t, lt in props:
                if lt is None:
                    pos += np.dtype(t).itemsize
                else:
                    c = int(np.frombuffer(data, bo + lt, 1, pos)[0])
                    pos += np.dtype(lt).itemsize + c * np.dtype(t).itemsize
    name, count, props = elems[vi]
    if any(lt is not None for _p, _t, lt in props):
        raise PlyError("list property in the vertex element")
    dt = np.dtype([(p, bo + t) for p, t, _lt in props])
    if len(data) - pos < count * dt.itemsize:
        raise PlyError("file ends before the last vertex")
    rec = np.frombuffer(data, dt, count, pos)
    return {p: rec[p] for p, _t, _lt in props}


def sh_degree_of(n_rest: int) -> int:
    for d in range(4):
        if n_rest == 3 * ((d + 1) ** 2 - 1):
            return d
    raise PlyError(f"{n_rest} f_rest properties")


def read(path) -> dict:
    with open(path, "rb") as f:
        data = f.read()
    fmt, elems, pos = read_header(data)
    if "vertex" not in [e[0] for e in elems]:
        raise PlyError("no vertex element")
    cols = _vertex_columns(fmt, elems, data, pos)
    n_rest = sum(1 for p in cols if p.startswith("f_rest_"))
    d = sh_degree_of(n_rest)
    m = (d + 1) ** 2 - 1

    def col(name):
        if name not in cols:
            raise PlyError("vertex property " + name + " missing")
        return np.asarray(cols[name]).astype(np.float32)

    n = len(cols["x"]) if "x" in cols else 0
    out = dict(
        means=np.stack([col(c) for c in ("x", "y", "z")], 1).reshape(n, 3),
        log_scales=np.stack([col(f"scale_{j}") for j in range(3)], 1).reshape(n, 3),
        quats=np.stack([col(f"rot_{j}") for j in range(4)], 1).reshape(n, 4),
        opacity_logits=col("opacity").reshape(n),
        sh=np.zeros((n, 16, 3), np.float32),
        sh_degree=d,
    )
    for c in range(3):
        out["sh"][:, 0, c] = col(f"f_dc_{c}")
        for k in range(1, m + 1):
            out["sh"][:, k, c] = col(f"f_rest_{c * m + k - 1}")
    return out
