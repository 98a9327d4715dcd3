"""PLY reading and model discovery (CPU): the PLY oracle against a
hand-written fixture and hand-built files, the library's reader
(tigas_ply_info / tigas_ply_read, host only) against the oracle, and the
registry's discovery of model folders (a registry without a context lists
models and refuses loads).  Section 5.1, PLY Model and Primitives and
Dynamic Multi-Model Runtime."""
import os
import struct

import numpy as np
import pytest

from oracle import ply as oply
from paper_2605_08699_amd import synth, tigas

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "ply_deg1_two_gaussians.ply")
KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")
F = np.float32


def _golden_expected():
    # written out by hand from the fixture's rows (not from any reader)
    sh = np.zeros((2, 16, 3), F)
    sh[0, 0] = (0.5, -0.5, 0.25)
    sh[0, 1], sh[0, 2], sh[0, 3] = (100, 103, 106), (101, 104, 107), (102, 105, 108)
    sh[1, 0] = (1, 2, 3)
    sh[1, 1], sh[1, 2], sh[1, 3] = (110, 113, 116), (111, 114, 117), (112, 115, 118)
    return dict(means=np.array([[1.5, -2.25, 3], [-0.125, 4, 8.5]], F),
                log_scales=np.array([[-3, -2.5, -2], [0.5, 0, -0.5]], F),
                quats=np.array([[0.9, 0.1, -0.2, 0.3], [1, 0, 0, 0]], F),
                opacity_logits=np.array([-1.5, 2.75], F), sh=sh)


def _same(a, b, keys=KEYS):
    for k in keys:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_oracle_reads_the_hand_written_fixture():
    o = oply.read(GOLDEN)
    assert o["sh_degree"] == 1
    _same(o, _golden_expected())


def test_library_reads_the_hand_written_fixture():
    assert tigas.ply_info(GOLDEN) == (2, 1)
    g = tigas.ply_read(GOLDEN)
    assert g["sh_degree"] == 1
    _same(g, _golden_expected())


# a file built property by property: every value is a function of the
# vertex index and the property name, so the expected arrays follow
# directly; an element with a list property precedes the vertices, the
# properties are out of the usual order and of several types
def _value(i, name):
    base = {"x": 1.0, "y": 2.0, "z": 3.0, "opacity": -0.75, "scale_0": -4.0, "scale_1": -3.5, "scale_2": -3.0,
            "rot_0": 0.5, "rot_1": -0.5, "rot_2": 0.25, "rot_3": 0.125, "f_dc_0": 0.3, "f_dc_1": -0.2,
            "f_dc_2": 0.1, "nx": 7.0, "red": 200.0}
    if name.startswith("f_rest_"):
        return 0.01 * int(name[7:]) - 0.5 * i
    return base[name] + 0.5 * i if name != "red" else 200.0 - i


def _hand_built(path, n, deg, byteorder="<", ascii_=False):
    m = (deg + 1) ** 2 - 1
    props = [("rot_3", "float", "f"), ("x", "double", "d"), ("red", "uchar", "B"), ("f_dc_2", "float", "f"),
             ("y", "float", "f"), ("z", "float", "f"), ("nx", "short", "h")]
    props += [(f"f_rest_{j}", "float", "f") for j in reversed(range(3 * m))]
    props += [("f_dc_0", "float", "f"), ("f_dc_1", "float", "f"), ("opacity", "double", "d"),
              ("scale_0", "float", "f"), ("scale_2", "float", "f"), ("scale_1", "float", "f"),
              ("rot_0", "float", "f"), ("rot_1", "float", "f"), ("rot_2", "float", "f")]
    fmt = "ascii" if ascii_ else ("binary_little_endian" if byteorder == "<" else "binary_big_endian")
    head = ["ply", f"format {fmt} 1.0", "comment built by the test", "element face 2",
            "property list uchar int vertex_indices", f"element vertex {n}"]
    head += [f"property {t} {p}" for p, t, _c in props] + ["element extra 1", "property float w", "end_header"]
    body = b""
    faces = [[0, 1, 2], [2, 3, 0, 1]]
    if ascii_:
        lines = [" ".join(str(v) for v in [len(f_)] + f_) for f_ in faces]
        for i in range(n):
            lines.append(" ".join(repr(float(_value(i, p))) if c in "fd" else str(int(_value(i, p)))
                                  for p, _t, c in props))
        lines.append("1.0")
        body = ("\n".join(lines) + "\n").encode()
    else:
        for f_ in faces:
            body += struct.pack(byteorder + "B" + "i" * len(f_), len(f_), *f_)
        for i in range(n):
            for p, _t, c in props:
                v = _value(i, p)
                body += struct.pack(byteorder + c, int(v) if c in "Bh" else v)
        body += struct.pack(byteorder + "f", 1.0)
    with open(path, "wb") as fh:
        fh.write(("\n".join(head) + "\n").encode() + body)
    want = dict(means=np.zeros((n, 3), F), log_scales=np.zeros((n, 3), F), quats=np.zeros((n, 4), F),
                opacity_logits=np.zeros(n, F), sh=np.zeros((n, 16, 3), F))
    for i in range(n):
        want["means"][i] = [_value(i, c) for c in "xyz"]
        want["log_scales"][i] = [_value(i, f"scale_{j}") for j in range(3)]
        want["quats"][i] = [_value(i, f"rot_{j}") for j in range(4)]
        want["opacity_logits"][i] = _value(i, "opacity")
        for c in range(3):
            want["sh"][i, 0, c] = _value(i, f"f_dc_{c}")
            for k in range(1, m + 1):
                want["sh"][i, k, c] = _value(i, f"f_rest_{c * m + k - 1}")
    return want


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
@pytest.mark.parametrize("enc", ["le", "be", "ascii"])
def test_hand_built_files(tmp_path, deg, enc):
    p = str(tmp_path / "m.ply")
    want = _hand_built(p, 5, deg, ">" if enc == "be" else "<", enc == "ascii")
    o = oply.read(p)
    assert o["sh_degree"] == deg
    _same(o, want)
    assert tigas.ply_info(p) == (5, deg)
    g = tigas.ply_read(p)
    _same(g, want)


@pytest.mark.parametrize("fmt", ["binary_little_endian", "binary_big_endian", "ascii"])
@pytest.mark.parametrize("deg", [0, 3])
def test_generator_files_round_trip(tmp_path, fmt, deg):
    sc = synth.scene_uniform(seed=11 + deg, n=700)
    sc.sh_degree = deg
    p = str(tmp_path / "s.ply")
    synth.write_ply(p, sc, fmt)
    o, g = oply.read(p), tigas.ply_read(p)
    m = (deg + 1) ** 2
    want = dict(means=sc.means, log_scales=sc.log_scales, quats=sc.quats, opacity_logits=sc.opacity_logits,
                sh=np.concatenate([sc.sh[:, :m], np.zeros((sc.n, 16 - m, 3), F)], 1))
    _same(o, want)
    _same(g, o)


def test_large_binary_file_matches_the_oracle(tmp_path):
    # more vertices than one read chunk of the library
    sc = synth.scene_uniform(seed=5, n=150_000)
    p = str(tmp_path / "big.ply")
    synth.write_ply(p, sc)
    _same(tigas.ply_read(p), oply.read(p))


def _write(path, text, body=b""):
    with open(path, "wb") as f:
        f.write(text.encode() + body)


def _header(props, n=1, fmt="binary_little_endian"):
    return f"ply\nformat {fmt} 1.0\nelement vertex {n}\n" + "".join(f"property float {p}\n" for p in props) + \
        "end_header\n"


BASE = ["x", "y", "z", "f_dc_0", "f_dc_1", "f_dc_2", "opacity", "scale_0", "scale_1", "scale_2",
        "rot_0", "rot_1", "rot_2", "rot_3"]


@pytest.mark.parametrize("case", ["not_ply", "no_end", "missing_prop", "bad_rest", "truncated", "vertex_list",
                                  "bad_format", "no_vertex"])
def test_malformed_files_are_rejected(tmp_path, case):
    p = str(tmp_path / "bad.ply")
    if case == "not_ply":
        _write(p, "hello\n")
    elif case == "no_end":
        _write(p, "ply\nformat ascii 1.0\nelement vertex 1\n")
    elif case == "missing_prop":
        _write(p, _header(BASE[:-1]), b"\0" * 52)
    elif case == "bad_rest":
        _write(p, _header(BASE + [f"f_rest_{j}" for j in range(10)]), b"\0" * 96)
    elif case == "truncated":
        _write(p, _header(BASE, n=3), b"\0" * (56 * 3 - 1))
    elif case == "vertex_list":
        _write(p, _header(BASE).replace("end_header", "property list uchar int idx\nend_header"), b"\0" * 57)
    elif case == "bad_format":
        _write(p, _header(BASE, fmt="binary_middle_endian"), b"\0" * 56)
    elif case == "no_vertex":
        _write(p, "ply\nformat ascii 1.0\nelement face 0\nproperty float a\nend_header\n")
    with pytest.raises(oply.PlyError):
        oply.read(p)
    with pytest.raises(tigas.TigasError) as e:
        tigas.ply_read(p)
    assert e.value.status == -1


def test_read_rejects_a_wrong_count(tmp_path):
    p = str(tmp_path / "s.ply")
    synth.write_ply(p, synth.scene_uniform(seed=1, n=10))
    buf = np.zeros(64 * 11, np.float32)
    L = tigas._registry_lib()
    assert L.tigas_ply_read(p.encode(), 11, *[tigas._ptr(buf)] * 5) == -1


def _model_tree(root):
    small = synth.scene_uniform(seed=2, n=50)
    big = synth.scene_uniform(seed=3, n=80)
    os.makedirs(root / "garden" / "point_cloud" / "iteration_7000")
    os.makedirs(root / "garden" / "point_cloud" / "iteration_30000")
    synth.write_ply(str(root / "garden" / "point_cloud" / "iteration_7000" / "point_cloud.ply"), small)
    synth.write_ply(str(root / "garden" / "point_cloud" / "iteration_30000" / "point_cloud.ply"), big)
    _write(str(root / "garden" / "preview.jpg"), "jpeg")
    os.makedirs(root / "room")
    synth.write_ply(str(root / "room" / "point_cloud.ply"), small)
    synth.write_ply(str(root / "room.ply"), big)  # same id as the folder: the folder wins
    os.makedirs(root / "bonsai")
    synth.write_ply(str(root / "bonsai" / "scene.ply"), small)
    synth.write_ply(str(root / "bonsai" / "z.ply"), big)
    os.makedirs(root / "empty")
    os.makedirs(root / "broken")
    _write(str(root / "broken" / "point_cloud.ply"), "not a ply\n")
    sc = synth.scene_uniform(seed=4, n=30)
    sc.sh_degree = 1
    synth.write_ply(str(root / "solo.ply"), sc, "ascii")
    _write(str(root / "solo.png"), "png")


def test_discovery(tmp_path):
    _model_tree(tmp_path)
    with tigas.Registry(None, str(tmp_path)) as reg:
        ms = reg.models()
        assert [m["id"] for m in ms] == ["bonsai", "garden", "room", "solo"]
        by = {m["id"]: m for m in ms}
        assert by["garden"]["ply_path"].endswith(os.path.join("iteration_30000", "point_cloud.ply"))
        assert by["garden"]["n"] == 80 and by["garden"]["sh_degree"] == 3
        assert by["garden"]["preview_path"].endswith(os.path.join("garden", "preview.jpg"))
        assert by["room"]["ply_path"].endswith(os.path.join("room", "point_cloud.ply")) and by["room"]["n"] == 50
        assert by["bonsai"]["ply_path"].endswith("scene.ply")
        assert by["solo"]["sh_degree"] == 1 and by["solo"]["preview_path"].endswith("solo.png")
        assert by["room"]["preview_path"] == ""
        for m in ms:
            assert not m["loaded"] and m["refs"] == 0 and m["loads"] == 0 and m["device_bytes"] == 0
        # no context: listing only
        with pytest.raises(tigas.TigasError):
            reg.acquire("garden")
        with pytest.raises(tigas.TigasError):
            reg.load("garden")
        assert reg.evict_idle() == 0
        assert not reg.info("garden")["loaded"]


def test_registry_arguments(tmp_path):
    with pytest.raises(tigas.TigasError):
        tigas.Registry(None, str(tmp_path / "missing"))
    with pytest.raises(tigas.TigasError):
        tigas.Registry(None, str(tmp_path), sweep_period_s=-1.0)
    with tigas.Registry(None, str(tmp_path)) as reg:
        assert len(reg) == 0
        with pytest.raises(tigas.TigasError):
            reg.acquire("nothing")


def test_sweeping_thread_stops_on_close(tmp_path):
    import time
    _model_tree(tmp_path)
    t0 = time.time()
    for _ in range(3):
        reg = tigas.Registry(None, str(tmp_path), idle_timeout_s=0.0, sweep_period_s=0.01)
        time.sleep(0.05)  # several sweeps over models that are not loaded
        assert len(reg) == 4 and reg.evict_idle() == 0
        reg.close()
    assert time.time() - t0 < 5.0
