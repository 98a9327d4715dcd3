"""The host code of libtigas under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the PLY reader (which parses untrusted files, on up to 16 host
threads) over valid, truncated, malformed and randomly corrupted files, a
discovery-only scene registry, and the latency-ABR controller.  The library's
sources are rebuilt with the sanitizers on their host code only (the GPU code
is compiled as usual and never runs here)."""
import hashlib
import os
import re
import shutil
import subprocess
import sys

import numpy as np
import pytest

from paper_2605_08699_amd import build as hipbuild
from paper_2605_08699_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2605_08699_amd", "csrc")
DRIVER = os.path.join(HERE, "host_sanitize", "driver.cpp")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _build(out_dir):
    srcs = [os.path.join(CSRC, s) for s in hipbuild.SOURCES] + [DRIVER]
    h = hashlib.sha1()
    for s in srcs + [os.path.join(ROOT, "include", "tigas.h"), os.path.join(CSRC, "tigas_internal.h")]:
        h.update(open(s, "rb").read())
    exe = os.path.join(out_dir, "driver_" + h.hexdigest()[:12])
    if os.path.exists(exe):
        return exe
    objs = []
    for s in srcs:
        o = os.path.join(out_dir, os.path.basename(s) + ".o")
        cmd = [hipbuild.HIPCC] + hipbuild.FLAGS + SAN + ["-O1", "-c", s, "-o", o]
        if s.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
        objs.append(o)
    subprocess.check_call([hipbuild.HIPCC, "--offload-arch=gfx950"] + SAN + ["-o", exe] + objs)
    return exe


def _fixtures(d):
    rng = np.random.default_rng(21)
    paths = []
    for i, (fmt, deg, n) in enumerate([("binary_little_endian", 3, 2000), ("binary_little_endian", 0, 1),
                                        ("binary_big_endian", 1, 300), ("ascii", 2, 40),
                                        ("binary_little_endian", 3, 300000)]):
        sc = synth.scene_uniform(seed=30 + i, n=n)
        sc.sh_degree = deg
        p = os.path.join(d, f"ok_{i}.ply")
        synth.write_ply(p, sc, fmt)
        paths.append(p)
    base = open(paths[0], "rb").read()
    head = base.index(b"end_header\n") + len(b"end_header\n")
    for i in range(40):  # corrupted copies: truncated, header bytes flipped, body garbage
        b = bytearray(base)
        kind = i % 4
        if kind == 0:
            b = b[: int(rng.integers(1, len(b)))]
        elif kind == 1:
            for _ in range(int(rng.integers(1, 6))):
                b[int(rng.integers(0, head))] = int(rng.integers(0, 256))
        elif kind == 2:
            k = int(rng.integers(head, len(b) - 64))
            b[k:k + 64] = rng.integers(0, 256, 64, dtype=np.uint8).tobytes()
        else:
            b = b[:head].replace(b"element vertex 2000", b"element vertex 99999999") + b[head:]
        p = os.path.join(d, f"bad_{i}.ply")
        open(p, "wb").write(bytes(b))
        paths.append(p)
    for name, text in (("empty.ply", b""), ("nul.ply", b"ply\0\0\0"),
                       ("huge_count.ply", b"ply\nformat ascii 1.0\nelement vertex 18446744073709551615\n"
                                          b"property float x\nend_header\n"),
                       ("neg_count.ply", b"ply\nformat ascii 1.0\nelement vertex -5\nend_header\n"),
                       ("ascii_short.ply", b"ply\nformat ascii 1.0\nelement vertex 2\nproperty float x\n"
                                           b"end_header\n1.0\n")):
        p = os.path.join(d, name)
        open(p, "wb").write(text)
        paths.append(p)
    # a registry root: one model folder and one root-level file
    os.makedirs(os.path.join(d, "root", "garden"))
    shutil.copy(paths[0], os.path.join(d, "root", "garden", "point_cloud.ply"))
    shutil.copy(paths[2], os.path.join(d, "root", "room.ply"))
    return paths


@pytest.mark.skipif(not os.path.exists(hipbuild.HIPCC), reason="hipcc not available")
def test_ply_reader_registry_and_abr_are_clean_under_asan_and_ubsan(tmp_path):
    cache = os.path.join("/tmp", "tigas_sanitize_build")
    os.makedirs(cache, exist_ok=True)
    exe = _build(cache)
    paths = _fixtures(str(tmp_path))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path / "root")] + paths, capture_output=True, env=env, timeout=600)
    out = (r.stdout + r.stderr).decode("utf-8", "replace")
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    m = re.search(r"files read (\d+), rejected (\d+)", out)
    assert m, out[-2000:]
    # the five valid files and the body-garbage copies parse; truncated and
    # malformed ones are rejected with an error status
    assert int(m.group(1)) >= 5 and int(m.group(2)) >= 20, m.group(0)
    for i in range(5):
        assert re.search(rf"ok_{i}\.ply: n=\d+ deg=\d status=0", out), i
    assert "model garden" in out and "model room" in out
