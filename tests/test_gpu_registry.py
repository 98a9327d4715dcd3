"""The scene registry on the GPU (needs an MI355X): lazy loading on first
access, reference counts, eviction after the inactivity timeout (on request
and by the registry's sweeping thread), one load for concurrent first
accesses, and frames of registry scenes identical to frames of the same
arrays loaded directly (read by the PLY oracle).  Section 4.1 and Section
5.1, Dynamic Multi-Model Runtime."""
import os
import threading
import time

import numpy as np
import pytest
import torch  # noqa: F401  (one HIP runtime: torch's, loaded before the library)

from oracle import ply as oply
from paper_2605_08699_amd import synth, tigas

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = tigas.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def root(tmp_path_factory):
    r = tmp_path_factory.mktemp("models")
    a = synth.scene_clusters(seed=21, n=30_000, n_clusters=8, surface_frac=0.3)
    b = synth.scene_uniform(seed=22, n=20_000)
    b.sh_degree = 1
    os.makedirs(r / "alpha")
    synth.write_ply(str(r / "alpha" / "point_cloud.ply"), a)
    synth.write_ply(str(r / "beta.ply"), b, "binary_big_endian")
    return r


def _render(ctx, scene, fmt):  # a host frame
    _, poses, _, _, _ = synth.c1_single_view()
    k = synth.fov_intrinsics(320, 240)
    return ctx.render(scene, poses[0], k, 320, 240, fmt=fmt)


class _Arrays:  # the oracle's arrays in the shape Context.load_scene takes
    def __init__(self, d):
        self.means, self.log_scales, self.quats = d["means"], d["log_scales"], d["quats"]
        self.opacity_logits, self.sh, self.sh_degree = d["opacity_logits"], d["sh"], d["sh_degree"]
        self.n = len(self.means)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_registry_scene_renders_like_a_direct_load(ctx, root, storage):
    with tigas.Registry(ctx, str(root), storage=storage) as reg:
        for mid, path in (("alpha", root / "alpha" / "point_cloud.ply"), ("beta", root / "beta.ply")):
            _say("registry render", mid, storage)
            s = reg.acquire(mid)
            direct = ctx.load_scene(_Arrays(oply.read(str(path))), storage=storage)
            assert reg.info(mid)["device_bytes"] == direct.bytes
            for fmt in ("rgb8", "f32"):
                a = _render(ctx, s, fmt)
                b = _render(ctx, direct, fmt)
                assert np.array_equal(a, b)
            assert _render(ctx, s, "rgb8").any()
            reg.release(s)
            direct.free()


def test_lazy_load_refcount_and_eviction(ctx, root):
    with tigas.Registry(ctx, str(root), idle_timeout_s=0.0) as reg:
        assert [m["id"] for m in reg.models()] == ["alpha", "beta"]
        assert not reg.info("alpha")["loaded"]
        _say("registry refcount")
        s1 = reg.acquire("alpha")
        i = reg.info("alpha")
        assert i["loaded"] and i["refs"] == 1 and i["loads"] == 1 and i["device_bytes"] > 0
        assert not reg.info("beta")["loaded"]  # only what was asked for
        s2 = reg.acquire("alpha")
        assert s2.handle.value == s1.handle.value and reg.info("alpha")["refs"] == 2
        reg.release(s1)
        assert reg.evict_idle() == 0  # still referenced
        _render(ctx, s2, "rgb8")
        reg.release(s2)
        with pytest.raises(tigas.TigasError):
            reg.release(s2)  # no reference left
        assert reg.evict_idle() == 1
        i = reg.info("alpha")
        assert not i["loaded"] and i["device_bytes"] == 0 and i["refs"] == 0
        with pytest.raises(tigas.TigasError):
            reg.release(s2)  # no longer resident
        s3 = reg.acquire("alpha")  # loaded again on the next access
        assert reg.info("alpha")["loads"] == 2
        _render(ctx, s3, "rgb8")
        reg.release(s3)
        reg.load("beta")  # explicit load: resident without a reference
        i = reg.info("beta")
        assert i["loaded"] and i["refs"] == 0 and i["sh_degree"] == 1
        assert reg.evict_idle() == 2


def test_idle_timeout(ctx, root):
    with tigas.Registry(ctx, str(root), idle_timeout_s=0.5) as reg:
        _say("registry idle timeout")
        s = reg.acquire("beta")
        reg.release(s)
        assert reg.evict_idle() == 0  # idle for less than the timeout
        time.sleep(0.7)
        assert reg.info("beta")["idle_s"] >= 0.5
        assert reg.evict_idle() == 1
    with tigas.Registry(ctx, str(root), idle_timeout_s=-1.0) as reg:
        reg.load("beta")
        assert reg.evict_idle() == 0  # never by age


def test_sweeping_thread(ctx, root):
    with tigas.Registry(ctx, str(root), idle_timeout_s=0.2, sweep_period_s=0.05) as reg:
        _say("registry sweeper")
        s = reg.acquire("alpha")
        time.sleep(0.6)
        assert reg.info("alpha")["loaded"]  # referenced: kept past the timeout
        reg.release(s)
        t0 = time.time()
        while reg.info("alpha")["loaded"] and time.time() - t0 < 5.0:
            time.sleep(0.05)
        assert not reg.info("alpha")["loaded"]
        assert time.time() - t0 >= 0.15


def test_concurrent_first_access_loads_once(ctx, root):
    with tigas.Registry(ctx, str(root)) as reg:
        _say("registry concurrent acquire")
        got, errs = [], []

        def take():
            try:
                got.append(reg.acquire("alpha"))
            except Exception as e:  # noqa: BLE001
                errs.append(e)

        ts = [threading.Thread(target=take) for _ in range(8)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        assert not errs
        assert len({s.handle.value for s in got}) == 1
        i = reg.info("alpha")
        assert i["loads"] == 1 and i["refs"] == 8
        for s in got:
            reg.release(s)
        assert reg.info("alpha")["refs"] == 0
