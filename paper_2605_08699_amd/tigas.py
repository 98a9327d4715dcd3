"""ctypes binding of libtigas.so (include/tigas.h): argument marshalling only.

Every step of a render runs in the HIP kernels of the library; this module
converts numpy arrays / torch tensors to pointers and structs.  There is no
CPU fallback: if the library is not built, loading it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtigas.so")

TIGAS_OK = 0
STATUS = {0: "OK", -1: "E_INVALID", -2: "E_OOM", -3: "E_DEVICE", -4: "E_BUFFER", -5: "E_BUDGET"}
ATTR = {"f32": 0, "f16": 1, "bf16": 2}
FMT = {"rgb8": 0, "f32": 1}


class TigasError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class SceneDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int),
                ("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p), ("quats_wxyz", ctypes.c_void_p),
                ("opacity_logits", ctypes.c_void_p), ("sh", ctypes.c_void_p),
                ("is_device", ctypes.c_int), ("storage", ctypes.c_int)]


class PoseC(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3)]


class IntrC(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class QualityC(ctypes.Structure):
    _fields_ = [("res_scale", ctypes.c_float), ("sh_degree", ctypes.c_int), ("fmt", ctypes.c_int),
                ("bg", ctypes.c_float * 3), ("tile_w", ctypes.c_int), ("tile_h", ctypes.c_int),
                ("batch_depth", ctypes.c_int), ("pixels_per_lane", ctypes.c_int)]


class FrameC(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("capacity", ctypes.c_size_t), ("is_device", ctypes.c_int),
                ("out_w", ctypes.c_int), ("out_h", ctypes.c_int)]


class StatsC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("visible", ctypes.c_int64), ("duplicates", ctypes.c_int64),
                ("fallbacks", ctypes.c_int64), ("tiles", ctypes.c_int64), ("sort_passes", ctypes.c_int64),
                ("rerenders", ctypes.c_int64), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("batch_depth", ctypes.c_int32), ("pixels_per_lane", ctypes.c_int32)]


class DebugC(ctypes.Structure):
    _fields_ = [("rec", ctypes.c_void_p), ("bbox", ctypes.c_void_p), ("zkey", ctypes.c_void_p),
                ("touched", ctypes.c_void_p), ("keys", ctypes.c_void_p), ("vals", ctypes.c_void_p),
                ("skeys", ctypes.c_void_p), ("svals", ctypes.c_void_p), ("ranges", ctypes.c_void_p),
                ("cap_dup", ctypes.c_int64), ("cap_tiles", ctypes.c_int64), ("n_dup", ctypes.c_int64),
                ("n_tiles", ctypes.c_int64)]


class StageC(ctypes.Structure):
    _fields_ = [("preprocess", ctypes.c_double), ("scan", ctypes.c_double), ("duplicate", ctypes.c_double),
                ("sort", ctypes.c_double), ("ranges", ctypes.c_double), ("blend", ctypes.c_double),
                ("frames", ctypes.c_int64)]


class KernelTimeC(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 120), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class AbrConfigC(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int), ("expected_bytes", ctypes.c_double * 8), ("t_target_s", ctypes.c_double),
                ("t_margin_s", ctypes.c_double), ("alpha", ctypes.c_double), ("history", ctypes.c_int),
                ("hold", ctypes.c_int), ("start_level", ctypes.c_int)]


# every symbol include/tigas.h declares
EXPORTS = ("tigas_context_create", "tigas_context_destroy", "tigas_scene_load", "tigas_scene_free",
           "tigas_scene_bytes", "tigas_render", "tigas_render_batch", "tigas_last_stats", "tigas_last_error",
           "tigas_render_debug", "tigas_selftest_wave_scan", "tigas_profile_stages", "tigas_stage_times",
           "tigas_count_blend_work", "tigas_set_graphs",
           "tigas_profile_kernels", "tigas_kernel_times", "tigas_render_submit", "tigas_render_wait",
           "tigas_jpeg_encode", "tigas_jpeg_max_bytes", "tigas_abr_default_config", "tigas_abr_create",
           "tigas_abr_destroy", "tigas_abr_observe", "tigas_abr_rate", "tigas_render_noalloc",
           "tigas_set_tile_binning", "tigas_set_tile_culling", "tigas_set_depth_passes")

_lib = None


def lib():
    """Load libtigas.so (built in-tree by build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2605_08699_amd.build.build()")
        try:  # one HIP runtime per process: torch's, loaded first so that the library binds to it
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        L.tigas_context_create.argtypes = [I, ctypes.POINTER(P)]
        L.tigas_context_destroy.argtypes = [P]
        L.tigas_context_destroy.restype = None
        L.tigas_scene_load.argtypes = [P, ctypes.POINTER(SceneDesc), ctypes.POINTER(P)]
        L.tigas_scene_free.argtypes = [P]
        L.tigas_scene_free.restype = None
        L.tigas_scene_bytes.argtypes = [P]
        L.tigas_scene_bytes.restype = ctypes.c_size_t
        L.tigas_render.argtypes = [P, ctypes.POINTER(PoseC), ctypes.POINTER(IntrC), I, I,
                                   ctypes.POINTER(QualityC), ctypes.POINTER(FrameC), P]
        L.tigas_render_debug.argtypes = [P, ctypes.POINTER(PoseC), ctypes.POINTER(IntrC), I, I,
                                         ctypes.POINTER(QualityC), ctypes.POINTER(FrameC), ctypes.POINTER(DebugC)]
        L.tigas_render_batch.argtypes = [ctypes.POINTER(P), ctypes.POINTER(PoseC), ctypes.POINTER(IntrC),
                                         ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(QualityC), I,
                                         ctypes.POINTER(FrameC), P]
        L.tigas_last_stats.argtypes = [P, ctypes.POINTER(StatsC)]
        L.tigas_last_error.argtypes = []
        L.tigas_last_error.restype = ctypes.c_char_p
        L.tigas_selftest_wave_scan.argtypes = [P, P, I]
        L.tigas_profile_stages.argtypes = [P, I]
        L.tigas_set_graphs.argtypes = [P, I]
        L.tigas_set_tile_binning.argtypes = [P, I]
        L.tigas_set_tile_culling.argtypes = [P, I]
        L.tigas_set_depth_passes.argtypes = [P, I]
        L.tigas_stage_times.argtypes = [P, ctypes.POINTER(StageC)]
        L.tigas_profile_kernels.argtypes = [P, I]
        L.tigas_render_submit.argtypes = [P, ctypes.POINTER(PoseC), ctypes.POINTER(IntrC), I, I,
                                          ctypes.POINTER(QualityC), ctypes.POINTER(FrameC), P, ctypes.POINTER(I64)]
        L.tigas_render_noalloc.argtypes = [P, ctypes.POINTER(PoseC), ctypes.POINTER(IntrC), I, I,
                                           ctypes.POINTER(QualityC), ctypes.POINTER(FrameC), P, P]
        L.tigas_render_wait.argtypes = [P, I64, ctypes.POINTER(StatsC), ctypes.POINTER(ctypes.c_float)]
        L.tigas_kernel_times.argtypes = [P, ctypes.POINTER(KernelTimeC), I, ctypes.POINTER(I)]
        L.tigas_jpeg_encode.argtypes = [P, P, I, I, I, P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t), P]
        L.tigas_jpeg_max_bytes.argtypes = [I, I]
        L.tigas_abr_default_config.argtypes = [ctypes.POINTER(AbrConfigC)]
        L.tigas_abr_default_config.restype = None
        L.tigas_abr_create.argtypes = [ctypes.POINTER(AbrConfigC), ctypes.POINTER(P)]
        L.tigas_abr_destroy.argtypes = [P]
        L.tigas_abr_destroy.restype = None
        L.tigas_abr_observe.argtypes = [P, ctypes.c_double, ctypes.c_double, I, ctypes.POINTER(I)]
        L.tigas_abr_rate.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
        L.tigas_jpeg_max_bytes.restype = ctypes.c_size_t
        L.tigas_count_blend_work.argtypes = [P, ctypes.POINTER(PoseC), ctypes.POINTER(IntrC), I, I,
                                             ctypes.POINTER(QualityC), ctypes.POINTER(FrameC),
                                             ctypes.POINTER(I64), ctypes.POINTER(I64)]
        for name in ("tigas_context_create", "tigas_scene_load", "tigas_render",
                     "tigas_render_debug",
                     "tigas_render_batch", "tigas_last_stats", "tigas_selftest_wave_scan", "tigas_profile_stages",
                     "tigas_stage_times", "tigas_count_blend_work", "tigas_set_graphs",
                     "tigas_profile_kernels", "tigas_kernel_times", "tigas_render_submit",
                     "tigas_render_wait", "tigas_jpeg_encode", "tigas_abr_create", "tigas_abr_observe",
                     "tigas_abr_rate"):
            getattr(L, name).restype = I
        _lib = L
    return _lib


def _check(status):
    if status != TIGAS_OK:
        raise TigasError(status, lib().tigas_last_error().decode())


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if isinstance(a, np.ndarray) else ctypes.c_void_p(int(a.data_ptr()))


def pose_c(pose) -> PoseC:
    p = PoseC()
    R = np.asarray(pose.R, np.float32).reshape(9)
    t = np.asarray(pose.t, np.float32).reshape(3)
    p.R[:] = [float(x) for x in R]
    p.t[:] = [float(x) for x in t]
    return p


def intr_c(k) -> IntrC:
    return IntrC(float(k.fx), float(k.fy), float(k.cx), float(k.cy))


def quality_c(res_scale=1.0, sh_degree=-1, fmt="rgb8", bg=(0.0, 0.0, 0.0), tile=None, batch_depth=None, ppl=None):
    """tile / batch_depth / ppl = None: chosen by the library's autotuner."""
    tile = (0, 0) if tile is None else tile
    batch_depth = 0 if batch_depth is None else batch_depth
    q = QualityC()
    q.pixels_per_lane = 0 if ppl is None else int(ppl)
    q.res_scale = float(res_scale)
    q.sh_degree = int(sh_degree)
    q.fmt = FMT[fmt]
    q.bg[:] = [float(x) for x in bg]
    q.tile_w, q.tile_h = int(tile[0]), int(tile[1])
    q.batch_depth = int(batch_depth)
    return q


def output_size(width, height, res_scale=1.0):
    s = float(np.float32(res_scale))
    return int(np.floor(width * s + 0.5)), int(np.floor(height * s + 0.5))


class Scene:
    """A resident scene.  ``borrowed`` scenes belong to a registry: free()
    only forgets the handle (the registry releases and unloads them)."""

    def __init__(self, ctx, handle, n, storage, borrowed=False):
        self.ctx = ctx
        self.handle = handle
        self.n = n
        self.storage = storage
        self.borrowed = borrowed

    @property
    def bytes(self) -> int:
        return int(lib().tigas_scene_bytes(self.handle))

    def free(self):
        if self.handle:
            if not self.borrowed:
                lib().tigas_scene_free(self.handle)
            self.handle = None


class Context:
    """A device, its stream and workspaces."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().tigas_context_create(int(device), ctypes.byref(h)))
        self.handle = h
        self._scenes = []

    def close(self):
        for s in self._scenes:
            s.free()
        self._scenes = []
        if self.handle:
            lib().tigas_context_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def load_scene(self, scene, storage: str = "f32") -> Scene:
        f32 = lambda a: np.ascontiguousarray(np.asarray(a, np.float32))
        arrs = [f32(scene.means), f32(scene.log_scales), f32(scene.quats), f32(scene.opacity_logits),
                f32(scene.sh).reshape(-1, 16, 3)]
        d = SceneDesc(scene.n, int(scene.sh_degree), *[ctypes.c_void_p(a.ctypes.data) for a in arrs], 0,
                      ATTR[storage])
        h = ctypes.c_void_p()
        _check(lib().tigas_scene_load(self.handle, ctypes.byref(d), ctypes.byref(h)))
        s = Scene(self, h, scene.n, storage)
        self._scenes.append(s)
        return s

    def stats(self) -> dict:
        st = StatsC()
        _check(lib().tigas_last_stats(self.handle, ctypes.byref(st)))
        return {f: int(getattr(st, f)) for f, _ in StatsC._fields_}

    def profile_stages(self, enable: bool = True):
        """Switch per-stage HIP-event timing on/off (resets the sums)."""
        _check(lib().tigas_profile_stages(self.handle, 1 if enable else 0))

    def stage_times(self) -> dict:
        st = StageC()
        _check(lib().tigas_stage_times(self.handle, ctypes.byref(st)))
        return {f: (int(getattr(st, f)) if f == "frames" else float(getattr(st, f))) for f, _ in StageC._fields_}

    def profile_kernels(self, enable: bool = True):
        """Switch per-launch HIP-event timing of every kernel on/off (clears the sums)."""
        _check(lib().tigas_profile_kernels(self.handle, 1 if enable else 0))

    def kernel_times(self) -> dict:
        """{kernel name: (launches, summed ms)} since profile_kernels(True)."""
        n = ctypes.c_int(0)
        _check(lib().tigas_kernel_times(self.handle, None, 0, ctypes.byref(n)))
        arr = (KernelTimeC * max(n.value, 1))()
        _check(lib().tigas_kernel_times(self.handle, arr, n.value, ctypes.byref(n)))
        return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n.value)}

    def set_graphs(self, enable: bool):
        """Capture/replay launch sequences as HIP graphs (default on)."""
        _check(lib().tigas_set_graphs(self.handle, 1 if enable else 0))

    def set_tile_binning(self, enable: bool):
        """Single views: tile digit by counting (True, the default) or by radix
        passes over the duplicates (False); identical lists either way."""
        _check(lib().tigas_set_tile_binning(self.handle, int(bool(enable))))

    def set_tile_culling(self, enable: bool):
        """Emit list entries only for tiles each Gaussian can reach (identical
        frames, fewer entries); off by default."""
        _check(lib().tigas_set_tile_culling(self.handle, int(bool(enable))))

    def set_depth_passes(self, passes: int):
        """Depth sort in three 9-bit passes with a four-pass fallback for
        frames too deep (3, the default) or always four 8-bit passes (4);
        identical frames either way."""
        _check(lib().tigas_set_depth_passes(self.handle, int(passes)))

    def count_blend_work(self, scene: Scene, pose, intr, width, height, res_scale=1.0, tile=None,
                         batch_depth=None, ppl=None):
        """(evaluations, contributions) of the blend kernel for one frame."""
        q = quality_c(res_scale, -1, "rgb8", (0, 0, 0), tile, batch_depth, ppl)
        ow, oh = output_size(width, height, res_scale)
        img = np.zeros((oh, ow, 3), np.uint8)
        fr = FrameC(ctypes.c_void_p(img.ctypes.data), img.nbytes, 0, 0, 0)
        e, c = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tigas_count_blend_work(scene.handle, ctypes.byref(pose_c(pose)), ctypes.byref(intr_c(intr)),
                                            int(width), int(height), ctypes.byref(q), ctypes.byref(fr),
                                            ctypes.byref(e), ctypes.byref(c)))
        return int(e.value), int(c.value)

    def render(self, scene: Scene, pose, intr, width, height, res_scale=1.0, fmt="rgb8", bg=(0, 0, 0),
               tile=None, batch_depth=None, sh_degree=-1, out=None, stream=None, ppl=None):
        """Render one frame.  ``out``: a torch tensor on the GPU (written in place)
        or None (a host numpy array is returned)."""
        q = quality_c(res_scale, sh_degree, fmt, bg, tile, batch_depth, ppl)
        ow, oh = output_size(width, height, res_scale)
        if out is None:
            out = np.zeros((oh, ow, 3), np.uint8 if fmt == "rgb8" else np.float32)
            fr = FrameC(ctypes.c_void_p(out.ctypes.data), out.nbytes, 0, 0, 0)
        else:
            fr = FrameC(ctypes.c_void_p(int(out.data_ptr())), out.numel() * out.element_size(), 1, 0, 0)
        st = ctypes.c_void_p(stream) if stream else None
        _check(lib().tigas_render(scene.handle, ctypes.byref(pose_c(pose)), ctypes.byref(intr_c(intr)),
                                  int(width), int(height), ctypes.byref(q), ctypes.byref(fr), st))
        return out

    def jpeg_encode(self, rgb, quality, out=None, stream=None):
        """Baseline JPEG of an RGB8 frame held in a GPU tensor [H, W, 3] (uint8).
        ``out``: a GPU uint8 tensor receiving the stream (sized by
        jpeg_max_bytes when None).  Returns (out, length)."""
        import torch
        assert rgb.is_cuda and rgb.dtype == torch.uint8 and rgb.dim() == 3 and rgb.shape[2] == 3
        assert rgb.is_contiguous()
        H, W = int(rgb.shape[0]), int(rgb.shape[1])
        if out is None:
            out = torch.empty(int(lib().tigas_jpeg_max_bytes(W, H)), dtype=torch.uint8, device=rgb.device)
        n = ctypes.c_size_t(0)
        st = ctypes.c_void_p(stream) if stream else None
        _check(lib().tigas_jpeg_encode(self.handle, ctypes.c_void_p(int(rgb.data_ptr())), W, H, int(quality),
                                       ctypes.c_void_p(int(out.data_ptr())), out.numel(), ctypes.byref(n), st))
        return out, int(n.value)

    def jpeg_bytes(self, rgb, quality, stream=None) -> bytes:
        """The JPEG stream of jpeg_encode copied to host memory."""
        out, n = self.jpeg_encode(rgb, quality, stream=stream)
        return out[:n].cpu().numpy().tobytes()

    def render_async(self, scene: Scene, pose, intr, width, height, out, res_scale=1.0, fmt="rgb8", bg=(0, 0, 0),
                     tile=None, batch_depth=None, sh_degree=-1, stream=None, ppl=None) -> int:
        """Launch one frame into the GPU tensor ``out`` and return its ticket
        without waiting; collect it with wait().  Two frames per stream may be
        in flight."""
        q = quality_c(res_scale, sh_degree, fmt, bg, tile, batch_depth, ppl)
        fr = FrameC(ctypes.c_void_p(int(out.data_ptr())), out.numel() * out.element_size(), 1, 0, 0)
        st = ctypes.c_void_p(stream) if stream else None
        t = ctypes.c_int64(0)
        _check(lib().tigas_render_submit(scene.handle, ctypes.byref(pose_c(pose)), ctypes.byref(intr_c(intr)),
                                         int(width), int(height), ctypes.byref(q), ctypes.byref(fr), st,
                                         ctypes.byref(t)))
        return int(t.value)

    def render_noalloc(self, scene: Scene, pose, intr, width, height, out, counters=None, res_scale=1.0,
                       fmt="rgb8", bg=(0, 0, 0), tile=None, batch_depth=None, sh_degree=-1, stream=None,
                       ppl=None) -> None:
        """Enqueue one frame into the GPU tensor ``out`` through the
        allocation-free entry point (buffers in the library's static device
        array) and return without waiting.  ``counters``: a GPU int32 tensor
        of 6 elements receiving (duplicates, visible, fallbacks, overflow, -, -)
        when the frame completes, or None."""
        q = quality_c(res_scale, sh_degree, fmt, bg, tile, batch_depth, ppl)
        fr = FrameC(ctypes.c_void_p(int(out.data_ptr())), out.numel() * out.element_size(), int(out.is_cuda), 0, 0)
        cp = None
        if counters is not None:
            assert counters.is_cuda and counters.numel() * counters.element_size() >= 24
            cp = ctypes.c_void_p(int(counters.data_ptr()))
        st = ctypes.c_void_p(stream) if stream else None
        _check(lib().tigas_render_noalloc(scene.handle, ctypes.byref(pose_c(pose)), ctypes.byref(intr_c(intr)),
                                          int(width), int(height), ctypes.byref(q), ctypes.byref(fr), cp, st))

    def wait(self, ticket: int) -> dict:
        """Wait for a submitted frame; its stats plus ``gpu_ms``."""
        st = StatsC()
        ms = ctypes.c_float(0.0)
        _check(lib().tigas_render_wait(self.handle, int(ticket), ctypes.byref(st), ctypes.byref(ms)))
        d = {f: int(getattr(st, f)) for f, _ in StatsC._fields_}
        d["gpu_ms"] = float(ms.value)
        return d

    def render_debug(self, scene: Scene, pose, intr, width, height, res_scale=1.0, fmt="f32", bg=(0, 0, 0),
                     tile=(16, 16), batch_depth=64, sh_degree=-1, cap_dup=None):
        """Render and return the intermediate stages (host arrays)."""
        q = quality_c(res_scale, sh_degree, fmt, bg, tile, batch_depth)
        ow, oh = output_size(width, height, res_scale)
        img = np.zeros((oh, ow, 3), np.uint8 if fmt == "rgb8" else np.float32)
        fr = FrameC(ctypes.c_void_p(img.ctypes.data), img.nbytes, 0, 0, 0)
        n = scene.n
        tiles_x = -(-ow // tile[0])
        tiles_y = -(-oh // tile[1])
        n_tiles = tiles_x * tiles_y
        if cap_dup is None:
            # first pass without the duplicate lists to learn D
            d0 = DebugC()
            _check(lib().tigas_render_debug(scene.handle, ctypes.byref(pose_c(pose)), ctypes.byref(intr_c(intr)),
                                            int(width), int(height), ctypes.byref(q), ctypes.byref(fr),
                                            ctypes.byref(d0)))
            cap_dup = int(d0.n_dup)
        out = dict(
            rec=np.zeros((n, 12), np.float32), bbox=np.zeros((n, 4), np.int32), zkey=np.zeros(n, np.uint32),
            touched=np.zeros(n, np.uint32), keys=np.zeros(cap_dup, np.uint64), vals=np.zeros(cap_dup, np.uint32),
            skeys=np.zeros(cap_dup, np.uint64), svals=np.zeros(cap_dup, np.uint32),
            ranges=np.zeros((n_tiles, 2), np.uint32))
        d = DebugC(*[ctypes.c_void_p(out[k].ctypes.data) for k in
                     ("rec", "bbox", "zkey", "touched", "keys", "vals", "skeys", "svals", "ranges")],
                   cap_dup, n_tiles, 0, 0)
        _check(lib().tigas_render_debug(scene.handle, ctypes.byref(pose_c(pose)), ctypes.byref(intr_c(intr)),
                                        int(width), int(height), ctypes.byref(q), ctypes.byref(fr), ctypes.byref(d)))
        D = int(d.n_dup)
        for k in ("keys", "vals", "skeys", "svals"):
            out[k] = out[k][:D]
        out["image"] = img
        out["n_dup"] = D
        out["tiles_x"], out["tiles_y"] = tiles_x, tiles_y
        return out

    def render_batch(self, scenes, poses, intrs, widths, heights, res_scales=None, fmt="rgb8", bg=(0, 0, 0),
                     tile=None, batch_depth=None, outs=None, stream=None, ppl=None):
        n = len(poses)
        res_scales = res_scales if res_scales is not None else [1.0] * n
        qs = (QualityC * n)(*[quality_c(res_scales[i], -1, fmt, bg, tile, batch_depth, ppl) for i in range(n)])
        frames = (FrameC * n)()
        results = []
        for i in range(n):
            ow, oh = output_size(widths[i], heights[i], res_scales[i])
            if outs is None:
                a = np.zeros((oh, ow, 3), np.uint8 if fmt == "rgb8" else np.float32)
                frames[i] = FrameC(ctypes.c_void_p(a.ctypes.data), a.nbytes, 0, 0, 0)
            else:
                a = outs[i]
                frames[i] = FrameC(ctypes.c_void_p(int(a.data_ptr())), a.numel() * a.element_size(), 1, 0, 0)
            results.append(a)
        hs = (ctypes.c_void_p * n)(*[s.handle.value if isinstance(s.handle, ctypes.c_void_p) else s.handle
                                     for s in scenes])
        ps = (PoseC * n)(*[pose_c(p) for p in poses])
        ks = (IntrC * n)(*[intr_c(k) for k in intrs])
        ws = (ctypes.c_int * n)(*[int(w) for w in widths])
        hh = (ctypes.c_int * n)(*[int(h) for h in heights])
        st = ctypes.c_void_p(stream) if stream else None
        _check(lib().tigas_render_batch(hs, ps, ks, ws, hh, qs, n, frames, st))
        return results


def selftest_wave_scan(values) -> np.ndarray:
    v = np.ascontiguousarray(np.asarray(values, np.uint32))
    out = np.zeros_like(v)
    _check(lib().tigas_selftest_wave_scan(ctypes.c_void_p(v.ctypes.data), ctypes.c_void_p(out.ctypes.data),
                                          int(v.size)))
    return out


# ------------------------------------------------------------------ serving

class ServerConfigC(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int), ("max_batch", ctypes.c_int), ("hbm_budget", ctypes.c_size_t),
                ("supersede", ctypes.c_int), ("tile_w", ctypes.c_int), ("tile_h", ctypes.c_int),
                ("batch_depth", ctypes.c_int), ("pixels_per_lane", ctypes.c_int), ("max_batch_pixels", ctypes.c_int64)]


class RequestC(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_void_p), ("pose", PoseC), ("intr", IntrC), ("width", ctypes.c_int),
                ("height", ctypes.c_int), ("q", QualityC), ("out", FrameC), ("client", ctypes.c_int),
                ("arrival_s", ctypes.c_double), ("jpeg_quality", ctypes.c_int), ("jpeg_out", ctypes.c_void_p),
                ("jpeg_capacity", ctypes.c_size_t)]


class CompletionC(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("client", ctypes.c_int), ("status", ctypes.c_int),
                ("arrival_s", ctypes.c_double), ("dispatch_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("batch_size", ctypes.c_int), ("jpeg_bytes", ctypes.c_int64)]


class ServerStatsC(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("admitted", "deferred", "superseded", "rendered", "failed", "batches",
                                              "max_batch_seen", "pending")]


SERVER_EXPORTS = ("tigas_server_create", "tigas_server_destroy", "tigas_server_submit", "tigas_server_poll",
                  "tigas_server_drain", "tigas_server_replay", "tigas_server_get_stats")
EXPORTS = EXPORTS + SERVER_EXPORTS


def _server_lib():
    L = lib()
    if not getattr(L, "_server_bound", False):
        P, I = ctypes.c_void_p, ctypes.c_int
        L.tigas_server_create.argtypes = [P, ctypes.POINTER(ServerConfigC), ctypes.POINTER(P)]
        L.tigas_server_destroy.argtypes = [P]
        L.tigas_server_destroy.restype = None
        L.tigas_server_submit.argtypes = [P, ctypes.POINTER(RequestC), ctypes.POINTER(ctypes.c_int64)]
        L.tigas_server_poll.argtypes = [P, ctypes.POINTER(CompletionC), I, ctypes.POINTER(I)]
        L.tigas_server_drain.argtypes = [P]
        L.tigas_server_replay.argtypes = [P, ctypes.POINTER(RequestC), I, ctypes.POINTER(CompletionC)]
        L.tigas_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStatsC)]
        for name in ("tigas_server_create", "tigas_server_submit", "tigas_server_poll", "tigas_server_drain",
                     "tigas_server_replay", "tigas_server_get_stats"):
            getattr(L, name).restype = I
        L._server_bound = True
    return L


def request_c(scene: Scene, pose, intr, width, height, out, client=0, arrival_s=0.0, res_scale=1.0, fmt="rgb8",
              bg=(0, 0, 0), jpeg_quality=0, jpeg_out=None):
    """One request; ``out`` is a torch GPU tensor or a host numpy array of the
    output frame (kept alive by the caller until it completes).  With
    ``jpeg_quality`` the frame is also encoded into the GPU uint8 tensor
    ``jpeg_out``."""
    r = RequestC()
    r.scene = scene.handle.value if isinstance(scene.handle, ctypes.c_void_p) else scene.handle
    r.pose = pose_c(pose)
    r.intr = intr_c(intr)
    r.width, r.height = int(width), int(height)
    r.q = quality_c(res_scale, -1, fmt, bg, (16, 32), 64)
    if isinstance(out, np.ndarray):
        r.out = FrameC(ctypes.c_void_p(out.ctypes.data), out.nbytes, 0, 0, 0)
    else:
        r.out = FrameC(ctypes.c_void_p(int(out.data_ptr())), out.numel() * out.element_size(), 1, 0, 0)
    r.client = int(client)
    r.arrival_s = float(arrival_s)
    if jpeg_quality:
        r.jpeg_quality = int(jpeg_quality)
        r.jpeg_out = ctypes.c_void_p(int(jpeg_out.data_ptr()))
        r.jpeg_capacity = jpeg_out.numel()
    return r


class Server:
    """Continuous-batching request loop of the library (tigas_server_*)."""

    def __init__(self, ctx: Context, slots=2, max_batch=64, hbm_budget=0, supersede=False, tile=(16, 32),
                 batch_depth=64, max_batch_pixels=0, ppl=0):
        L = _server_lib()
        cfg = ServerConfigC(int(slots), int(max_batch), int(hbm_budget), 1 if supersede else 0, int(tile[0]),
                            int(tile[1]), int(batch_depth), int(ppl), int(max_batch_pixels))
        h = ctypes.c_void_p()
        _check(L.tigas_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            _server_lib().tigas_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def submit(self, req: RequestC) -> int:
        i = ctypes.c_int64()
        _check(_server_lib().tigas_server_submit(self.handle, ctypes.byref(req), ctypes.byref(i)))
        return int(i.value)

    def drain(self):
        _check(_server_lib().tigas_server_drain(self.handle))

    def poll(self, max_n=4096):
        buf = (CompletionC * max_n)()
        n = ctypes.c_int()
        _check(_server_lib().tigas_server_poll(self.handle, buf, max_n, ctypes.byref(n)))
        return [_completion_dict(buf[i]) for i in range(n.value)]

    def replay(self, reqs):
        n = len(reqs)
        arr = (RequestC * n)(*reqs)
        out = (CompletionC * n)()
        _check(_server_lib().tigas_server_replay(self.handle, arr, n, out))
        return [_completion_dict(out[i]) for i in range(n)]

    def stats(self) -> dict:
        st = ServerStatsC()
        _check(_server_lib().tigas_server_get_stats(self.handle, ctypes.byref(st)))
        return {f: int(getattr(st, f)) for f, _ in ServerStatsC._fields_}


def _completion_dict(c):
    return dict(id=int(c.id), client=int(c.client), status=int(c.status), arrival_s=c.arrival_s,
                dispatch_s=c.dispatch_s, done_s=c.done_s, batch_size=int(c.batch_size),
                jpeg_bytes=int(c.jpeg_bytes))


class ABR:
    """The library's latency ABR controller (tigas_abr_*): observe() takes a
    completed request's payload bytes and download seconds and returns the
    level of the next request (0 = the smallest rung)."""

    def __init__(self, expected_bytes=None, t_target=None, t_margin=None, alpha=None, history=None, hold=None,
                 level=None):
        L = lib()
        cfg = AbrConfigC()
        L.tigas_abr_default_config(ctypes.byref(cfg))
        if expected_bytes is not None:
            cfg.n_levels = len(expected_bytes)
            for i, b in enumerate(expected_bytes):
                cfg.expected_bytes[i] = float(b)
        for name, v in (("t_target_s", t_target), ("t_margin_s", t_margin), ("alpha", alpha)):
            if v is not None:
                setattr(cfg, name, float(v))
        for name, v in (("history", history), ("hold", hold), ("start_level", level)):
            if v is not None:
                setattr(cfg, name, int(v))
        h = ctypes.c_void_p()
        _check(L.tigas_abr_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h

    def observe(self, nbytes, seconds, rapid_pan=False) -> int:
        lv = ctypes.c_int()
        _check(lib().tigas_abr_observe(self.handle, float(nbytes), float(seconds), 1 if rapid_pan else 0,
                                       ctypes.byref(lv)))
        return int(lv.value)

    @property
    def rate_kbps(self) -> float:
        r = ctypes.c_double()
        _check(lib().tigas_abr_rate(self.handle, ctypes.byref(r)))
        return float(r.value)

    def close(self):
        if self.handle:
            lib().tigas_abr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RegistryConfigC(ctypes.Structure):
    _fields_ = [("idle_timeout_s", ctypes.c_double), ("sweep_period_s", ctypes.c_double), ("storage", ctypes.c_int)]


class ModelInfoC(ctypes.Structure):
    _fields_ = [("id", ctypes.c_char_p), ("ply_path", ctypes.c_char_p), ("preview_path", ctypes.c_char_p),
                ("n", ctypes.c_int64), ("sh_degree", ctypes.c_int), ("loaded", ctypes.c_int), ("refs", ctypes.c_int),
                ("loads", ctypes.c_int64), ("device_bytes", ctypes.c_size_t), ("idle_s", ctypes.c_double)]


REGISTRY_EXPORTS = ("tigas_ply_info", "tigas_ply_read", "tigas_registry_default_config", "tigas_registry_create",
                    "tigas_registry_destroy", "tigas_registry_count", "tigas_registry_info", "tigas_registry_acquire",
                    "tigas_registry_load", "tigas_registry_release", "tigas_registry_evict_idle")
EXPORTS = EXPORTS + REGISTRY_EXPORTS


def _registry_lib():
    L = lib()
    if not getattr(L, "_registry_bound", False):
        P, I, I64, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_char_p
        L.tigas_ply_info.argtypes = [S, ctypes.POINTER(I64), ctypes.POINTER(I)]
        L.tigas_ply_read.argtypes = [S, I64, P, P, P, P, P]
        L.tigas_registry_default_config.argtypes = [ctypes.POINTER(RegistryConfigC)]
        L.tigas_registry_default_config.restype = None
        L.tigas_registry_create.argtypes = [P, S, ctypes.POINTER(RegistryConfigC), ctypes.POINTER(P)]
        L.tigas_registry_destroy.argtypes = [P]
        L.tigas_registry_destroy.restype = None
        L.tigas_registry_count.argtypes = [P]
        L.tigas_registry_count.restype = I64
        L.tigas_registry_info.argtypes = [P, I64, ctypes.POINTER(ModelInfoC)]
        L.tigas_registry_acquire.argtypes = [P, S, ctypes.POINTER(P)]
        L.tigas_registry_load.argtypes = [P, S]
        L.tigas_registry_release.argtypes = [P, P]
        L.tigas_registry_evict_idle.argtypes = [P, ctypes.POINTER(I)]
        for name in ("tigas_ply_info", "tigas_ply_read", "tigas_registry_create", "tigas_registry_info",
                     "tigas_registry_acquire", "tigas_registry_load", "tigas_registry_release",
                     "tigas_registry_evict_idle"):
            getattr(L, name).restype = I
        L._registry_bound = True
    return L


def ply_info(path) -> tuple:
    """(vertex count, SH degree) of a 3DGS PLY file (tigas_ply_info; host only)."""
    L = _registry_lib()
    n, d = ctypes.c_int64(), ctypes.c_int()
    _check(L.tigas_ply_info(os.fsencode(path), ctypes.byref(n), ctypes.byref(d)))
    return int(n.value), int(d.value)


def ply_read(path) -> dict:
    """The scene arrays of a 3DGS PLY file as read by the library
    (tigas_ply_read; host only): means, log_scales, quats (w, x, y, z),
    opacity_logits, sh [n, 16, 3] and sh_degree."""
    L = _registry_lib()
    n, deg = ply_info(path)
    out = dict(means=np.empty((n, 3), np.float32), log_scales=np.empty((n, 3), np.float32),
               quats=np.empty((n, 4), np.float32), opacity_logits=np.empty(n, np.float32),
               sh=np.empty((n, 16, 3), np.float32))
    _check(L.tigas_ply_read(os.fsencode(path), n, *[_ptr(out[k]) for k in
                                                   ("means", "log_scales", "quats", "opacity_logits", "sh")]))
    out["sh_degree"] = deg
    return out


class Registry:
    """The library's scene registry (tigas_registry_*): models found under
    ``root`` at creation, loaded on first access, reference-counted while
    acquired and unloaded by sweeps once idle for ``idle_timeout_s``.  With
    ``ctx`` None it only lists the models.  Close it before its context."""

    def __init__(self, ctx, root, idle_timeout_s=300.0, sweep_period_s=0.0, storage="f32"):
        L = _registry_lib()
        cfg = RegistryConfigC(float(idle_timeout_s), float(sweep_period_s), ATTR[storage])
        h = ctypes.c_void_p()
        _check(L.tigas_registry_create(ctx.handle if ctx is not None else None, os.fsencode(root),
                                       ctypes.byref(cfg), ctypes.byref(h)))
        self.ctx = ctx
        self.storage = storage
        self.handle = h

    def __len__(self):
        return int(_registry_lib().tigas_registry_count(self.handle))

    def _info(self, i) -> dict:
        c = ModelInfoC()
        _check(_registry_lib().tigas_registry_info(self.handle, int(i), ctypes.byref(c)))
        return dict(id=c.id.decode(), ply_path=c.ply_path.decode(), preview_path=c.preview_path.decode(),
                    n=int(c.n), sh_degree=int(c.sh_degree), loaded=bool(c.loaded), refs=int(c.refs),
                    loads=int(c.loads), device_bytes=int(c.device_bytes), idle_s=float(c.idle_s))

    def models(self) -> list:
        return [self._info(i) for i in range(len(self))]

    def info(self, model_id) -> dict:
        for m in self.models():
            if m["id"] == model_id:
                return m
        raise KeyError(model_id)

    def acquire(self, model_id) -> Scene:
        """The resident scene of model ``model_id`` (loaded now if needed),
        with a reference held until ``release``."""
        h = ctypes.c_void_p()
        _check(_registry_lib().tigas_registry_acquire(self.handle, model_id.encode(), ctypes.byref(h)))
        return Scene(self.ctx, h, self.info(model_id)["n"], self.storage, borrowed=True)

    def release(self, scene: Scene):
        _check(_registry_lib().tigas_registry_release(self.handle, scene.handle))

    def load(self, model_id):
        _check(_registry_lib().tigas_registry_load(self.handle, model_id.encode()))

    def evict_idle(self) -> int:
        k = ctypes.c_int()
        _check(_registry_lib().tigas_registry_evict_idle(self.handle, ctypes.byref(k)))
        return int(k.value)

    def close(self):
        if self.handle:
            _registry_lib().tigas_registry_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
