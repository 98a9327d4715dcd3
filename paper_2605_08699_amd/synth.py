"""Seeded synthetic inputs: Gaussian scenes, camera poses, trajectories, client traces.

This module only draws random inputs; it holds none of the rasterizer's
arithmetic, so both the HIP path and the CPU oracle can be fed from it.

The paper renders real 3DGS scenes (Kerbl et al. 2023) along recorded 6DoF
head-movement traces (Section 6, evaluation setup); neither is available here.
The generators below stand in for them with the per-Gaussian attribute layout
of Section 5.1 (centres, log-scales, unit quaternions, opacity logits,
SH coefficients of shape N x 16 x 3) and smooth random-walk camera paths.

Conventions
-----------
* A pose is ``(R, t)``: ``R`` is the camera-to-world rotation (columns are the
  camera axes in world coordinates, OpenCV axes: x right, y down, z forward),
  ``t`` the camera centre.  The world-to-camera transform is
  ``[R^T, -R^T t]`` (Section 5.1, rendering engine).
* ``N(m, s)`` below takes ``s`` as the standard deviation.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

F32 = np.float32

# bitrate-ladder resolution scales of 1920x1080 used by the batched and
# serving workloads (the paper's Table 1 ladder is exactly these four scales)
RUNG_SCALES = (0.25, 0.5, 0.75, 1.0)


@dataclasses.dataclass
class Scene:
    means: np.ndarray            # f32 [N,3]
    log_scales: np.ndarray       # f32 [N,3]
    quats: np.ndarray            # f32 [N,4]  (w, x, y, z), not necessarily unit length
    opacity_logits: np.ndarray   # f32 [N]
    sh: np.ndarray               # f32 [N,16,3] coefficient-major
    sh_degree: int = 3

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        return Scene(self.means[idx].copy(), self.log_scales[idx].copy(), self.quats[idx].copy(),
                     self.opacity_logits[idx].copy(), self.sh[idx].copy(), self.sh_degree)

    def permuted(self, perm) -> "Scene":
        return self.subset(np.asarray(perm))


@dataclasses.dataclass
class Pose:
    R: np.ndarray   # f32 [3,3] camera -> world
    t: np.ndarray   # f32 [3] camera centre


@dataclasses.dataclass
class Intrinsics:
    fx: float
    fy: float
    cx: float
    cy: float


def fov_intrinsics(width: int, height: int, hfov_deg: float = 60.0) -> Intrinsics:
    """Pinhole intrinsics with the given horizontal field of view, square pixels,
    principal point at the image centre."""
    f = width / (2.0 * math.tan(math.radians(hfov_deg) / 2.0))
    return Intrinsics(float(F32(f)), float(F32(f)), width / 2.0, height / 2.0)


def _normalize(v, axis=-1):
    return v / np.linalg.norm(v, axis=axis, keepdims=True)


def _quat_to_mat(q):
    """(w,x,y,z) unit quaternions [K,4] -> rotation matrices [K,3,3] (float64)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    m = np.empty((q.shape[0], 3, 3))
    m[:, 0, 0] = 1 - 2 * (y * y + z * z)
    m[:, 0, 1] = 2 * (x * y - w * z)
    m[:, 0, 2] = 2 * (x * z + w * y)
    m[:, 1, 0] = 2 * (x * y + w * z)
    m[:, 1, 1] = 1 - 2 * (x * x + z * z)
    m[:, 1, 2] = 2 * (y * z - w * x)
    m[:, 2, 0] = 2 * (x * z - w * y)
    m[:, 2, 1] = 2 * (y * z + w * x)
    m[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return m


def _mat_to_quat(m):
    """Rotation matrices [K,3,3] -> (w,x,y,z) quaternions [K,4] (Shepperd's method)."""
    k = m.shape[0]
    q = np.empty((k, 4))
    tr = m[:, 0, 0] + m[:, 1, 1] + m[:, 2, 2]
    cands = np.stack([tr, m[:, 0, 0], m[:, 1, 1], m[:, 2, 2]], axis=1)
    which = np.argmax(cands, axis=1)
    for c in range(4):
        sel = which == c
        if not np.any(sel):
            continue
        a = m[sel]
        if c == 0:
            s = np.sqrt(1.0 + tr[sel]) * 2
            q[sel] = np.stack([0.25 * s, (a[:, 2, 1] - a[:, 1, 2]) / s,
                               (a[:, 0, 2] - a[:, 2, 0]) / s, (a[:, 1, 0] - a[:, 0, 1]) / s], 1)
        elif c == 1:
            s = np.sqrt(1.0 + a[:, 0, 0] - a[:, 1, 1] - a[:, 2, 2]) * 2
            q[sel] = np.stack([(a[:, 2, 1] - a[:, 1, 2]) / s, 0.25 * s,
                               (a[:, 0, 1] + a[:, 1, 0]) / s, (a[:, 0, 2] + a[:, 2, 0]) / s], 1)
        elif c == 2:
            s = np.sqrt(1.0 + a[:, 1, 1] - a[:, 0, 0] - a[:, 2, 2]) * 2
            q[sel] = np.stack([(a[:, 0, 2] - a[:, 2, 0]) / s, (a[:, 0, 1] + a[:, 1, 0]) / s,
                               0.25 * s, (a[:, 1, 2] + a[:, 2, 1]) / s], 1)
        else:
            s = np.sqrt(1.0 + a[:, 2, 2] - a[:, 0, 0] - a[:, 1, 1]) * 2
            q[sel] = np.stack([(a[:, 1, 0] - a[:, 0, 1]) / s, (a[:, 0, 2] + a[:, 2, 0]) / s,
                               (a[:, 1, 2] + a[:, 2, 1]) / s, 0.25 * s], 1)
    return q


def _attributes(rng, n, sh_degree=3):
    """Per-Gaussian attributes shared by every synthetic workload:
    log-scales N(-4, 0.5) per axis, uniform random unit quaternions,
    opacity logits N(0, 1.5), SH DC N(0, 0.5) and higher bands N(0, 0.05)."""
    log_scales = rng.normal(-4.0, 0.5, size=(n, 3)).astype(F32)
    quats = _normalize(rng.normal(size=(n, 4))).astype(F32)
    opac = rng.normal(0.0, 1.5, size=n).astype(F32)
    sh = np.empty((n, 16, 3), dtype=F32)
    sh[:, 0, :] = rng.normal(0.0, 0.5, size=(n, 3))
    sh[:, 1:, :] = rng.normal(0.0, 0.05, size=(n, 15, 3))
    if sh_degree < 3:
        sh[:, (sh_degree + 1) ** 2:, :] = 0.0
    return log_scales, quats, opac, sh


def scene_uniform(seed: int = 1, n: int = 20000, half_extent: float = 1.0) -> Scene:
    """Centres uniform in [-h, h]^3 (the 20k-Gaussian single-view workload)."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-half_extent, half_extent, size=(n, 3)).astype(F32)
    ls, q, o, sh = _attributes(rng, n)
    return Scene(means, ls, q, o, sh, 3)


def _sample_in_box(draw, n, lo=-5.0, hi=5.0):
    out = np.empty((0, 3))
    extra = []
    while out.shape[0] < n:
        pts, aux = draw(max(1024, int((n - out.shape[0]) * 1.3)))
        keep = np.all((pts >= lo) & (pts <= hi), axis=1)
        out = np.concatenate([out, pts[keep]])
        extra.append(aux[keep] if aux is not None else None)
    if extra[0] is not None:
        aux_all = np.concatenate(extra)[:n]
    else:
        aux_all = None
    return out[:n], aux_all


def scene_clusters(seed: int, n: int, n_clusters: int, surface_frac: float = 0.0) -> Scene:
    """Centres drawn from an equal-weight mixture of anisotropic Gaussian clusters
    inside [-5,5]^3 (cluster centre U[-5,5]^3, per-axis std U[0.2,1.5], random
    orientation; samples outside the box are redrawn).  A fraction
    ``surface_frac`` are flattened surface splats lying on the cluster
    ellipsoids at Mahalanobis radius 2, oriented with their thin axis along the
    ellipsoid normal (random spin about it), log-scales (N(-4,0.5), N(-4,0.5),
    N(-7,0.3))."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-5.0, 5.0, size=(n_clusters, 3))
    sig = rng.uniform(0.2, 1.5, size=(n_clusters, 3))
    rot = _quat_to_mat(_normalize(rng.normal(size=(n_clusters, 4))))
    n_surf = int(round(n * surface_frac))
    n_vol = n - n_surf

    def draw_vol(m):
        k = rng.integers(0, n_clusters, size=m)
        xi = rng.normal(size=(m, 3)) * sig[k]
        return centres[k] + np.einsum("kij,kj->ki", rot[k], xi), None

    vol, _ = _sample_in_box(draw_vol, n_vol)
    ls, q, o, sh = _attributes(rng, n)
    means = np.empty((n, 3))
    means[:n_vol] = vol
    if n_surf:
        def draw_surf(m):
            k = rng.integers(0, n_clusters, size=m)
            u = _normalize(rng.normal(size=(m, 3)))
            p = centres[k] + np.einsum("kij,kj->ki", rot[k], 2.0 * sig[k] * u)
            nrm = _normalize(np.einsum("kij,kj->ki", rot[k], u / sig[k]))
            return p, nrm

        surf, nrm = _sample_in_box(draw_surf, n_surf)
        means[n_vol:] = surf
        r = _normalize(rng.normal(size=(n_surf, 3)))
        t1 = _normalize(np.cross(nrm, r))
        t2 = np.cross(nrm, t1)
        frame = np.stack([t1, t2, nrm], axis=2)          # columns = local axes
        q[n_vol:] = _mat_to_quat(frame).astype(F32)
        ls[n_vol:, 0] = rng.normal(-4.0, 0.5, size=n_surf)
        ls[n_vol:, 1] = rng.normal(-4.0, 0.5, size=n_surf)
        ls[n_vol:, 2] = rng.normal(-7.0, 0.3, size=n_surf)
    perm = rng.permutation(n)
    return Scene(means[perm].astype(F32), ls[perm], q[perm], o[perm], sh[perm], 3)


def _rodrigues(axis, ang):
    a = axis / np.linalg.norm(axis)
    k = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * k + (1 - math.cos(ang)) * (k @ k)


def _orthonormalize(R):
    u, _, vt = np.linalg.svd(R)
    return u @ vt


def look_at(position, target=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Camera-to-world rotation whose forward (z) axis points at ``target`` and
    whose down (y) axis is as close to world +y as possible."""
    f = _normalize(np.asarray(target, float) - np.asarray(position, float))
    x = np.cross([0.0, 1.0, 0.0], f)
    if np.linalg.norm(x) < 1e-8:
        x = np.cross([0.0, 0.0, 1.0], f)
    x = _normalize(x)
    y = np.cross(f, x)
    return np.stack([x, y, f], axis=1)


def trajectory(seed: int, n_poses: int = 300, t0=(0.0, 0.0, -8.0), R0=None,
               step: float = 0.02, rot_deg: float = 0.5, drift: float = 0.2,
               keep_in_view_deg: float = 30.0) -> list:
    """Smooth 6DoF random walk: per step the camera moves ``step`` units along a
    unit velocity that drifts (v <- normalise(v + drift*xi)) and rotates by
    ``rot_deg`` about an axis (camera frame) that drifts the same way; when the
    forward axis is more than ``keep_in_view_deg`` off the direction to the
    origin, the rotation axis is turned to swing the view back toward it."""
    rng = np.random.default_rng(seed)
    R = np.eye(3) if R0 is None else np.asarray(R0, float)
    t = np.asarray(t0, float).copy()
    v = _normalize(rng.normal(size=3))
    a = _normalize(rng.normal(size=3))
    ang = math.radians(rot_deg)
    keep = math.radians(keep_in_view_deg)
    poses = []
    for _ in range(n_poses):
        poses.append(Pose(R.astype(F32), t.astype(F32)))
        v = _normalize(v + drift * rng.normal(size=3))
        a = _normalize(a + drift * rng.normal(size=3))
        t = t + step * v
        fwd = R[:, 2]
        to_o = -t / max(np.linalg.norm(t), 1e-12)
        off = math.acos(float(np.clip(fwd @ to_o, -1.0, 1.0)))
        if off > keep:
            ax_w = np.cross(fwd, to_o)
            if np.linalg.norm(ax_w) > 1e-12:
                a = _normalize(R.T @ ax_w)
        R = _orthonormalize(R @ _rodrigues(a, ang))
    return poses


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def c1_single_view():
    """20k Gaussians in [-1,1]^3, one pose at (0,0,-3) looking at the origin, 256x256, 60 deg FoV."""
    scene = scene_uniform(seed=1, n=20000)
    pose = Pose(np.eye(3, dtype=F32), np.array([0.0, 0.0, -3.0], F32))
    return scene, [pose], fov_intrinsics(256, 256), 256, 256


def c2_scene(n: int = 1_000_000):
    return scene_clusters(seed=2, n=n, n_clusters=32, surface_frac=0.0)


def c2_trajectory(n_poses: int = 300):
    return trajectory(seed=102, n_poses=n_poses)


def c3_scene(n: int = 3_000_000):
    return scene_clusters(seed=3, n=n, n_clusters=64, surface_frac=0.4)


def c3_trajectory(n_poses: int = 300):
    return trajectory(seed=103, n_poses=n_poses)


def c4_views(traj=None):
    """32 poses (trajectory indices 0, 9, ..., 279) at rungs 0.25/0.5/0.75/1.0 of 1920x1080."""
    traj = traj if traj is not None else c3_trajectory(300)
    poses = [traj[i] for i in range(0, 280, 9)][:32]
    scales = [RUNG_SCALES[i % 4] for i in range(32)]
    return poses, scales


@dataclasses.dataclass
class ClientTrace:
    scene_id: int
    arrivals_s: np.ndarray      # request arrival times (seconds from start)
    rungs: np.ndarray           # resolution scale per request
    poses: list                 # one pose per request


def serving_clients(n_clients: int = 64, rate_hz: float = 60.0, duration_s: float = 11.0,
                    n_scenes: int = 4) -> list:
    """Open-loop client traces: client c renders scene c mod 4, walks its own
    trajectory (seed 1000+c) starting on a radius-8 sphere looking at the origin,
    sends requests with exponential gaps of mean 1/rate (seed 2000+c) at a
    uniformly random rung (seed 3000+c)."""
    clients = []
    for c in range(n_clients):
        rs = np.random.default_rng(1000 + c)
        start = 8.0 * _normalize(rs.normal(size=3))
        gaps = np.random.default_rng(2000 + c).exponential(1.0 / rate_hz, size=int(duration_s * rate_hz * 2) + 16)
        arr = np.cumsum(gaps)
        arr = arr[arr < duration_s]
        rungs = np.random.default_rng(3000 + c).choice(np.array(RUNG_SCALES), size=arr.shape[0])
        poses = trajectory(seed=1000 + c, n_poses=arr.shape[0], t0=start, R0=look_at(start))
        clients.append(ClientTrace(c % n_scenes, arr, rungs, poses))
    return clients


def serving_scenes(sizes=(500_000, 1_000_000, 3_000_000, 6_000_000), seeds=(50, 51, 52, 53)):
    return [scene_clusters(seed=s, n=n, n_clusters=64, surface_frac=0.4) for n, s in zip(sizes, seeds)]


def write_ply(path, scene: Scene, fmt: str = "binary_little_endian") -> None:
    """Writes ``scene`` as a 3DGS model file (the vertex layout of the 3DGS
    training output: x y z nx ny nz f_dc_0..2 f_rest_* opacity scale_0..2
    rot_0..3, FP32, normals zero; f_rest channel-major), in ``fmt``: ascii,
    binary_little_endian or binary_big_endian."""
    d = int(scene.sh_degree)
    m = (d + 1) ** 2 - 1
    names = ["x", "y", "z", "nx", "ny", "nz", "f_dc_0", "f_dc_1", "f_dc_2"]
    names += [f"f_rest_{j}" for j in range(3 * m)]
    names += ["opacity", "scale_0", "scale_1", "scale_2", "rot_0", "rot_1", "rot_2", "rot_3"]
    n = scene.n
    rest = np.asarray(scene.sh, F32)[:, 1:m + 1, :].transpose(0, 2, 1).reshape(n, 3 * m)  # [n, channel, coef]
    cols = np.concatenate([np.asarray(scene.means, F32), np.zeros((n, 3), F32), np.asarray(scene.sh, F32)[:, 0, :],
                           rest, np.asarray(scene.opacity_logits, F32).reshape(n, 1),
                           np.asarray(scene.log_scales, F32), np.asarray(scene.quats, F32)], 1)
    head = "ply\nformat %s 1.0\nelement vertex %d\n" % (fmt, n)
    head += "".join("property float %s\n" % p for p in names) + "end_header\n"
    with open(path, "wb") as f:
        f.write(head.encode("ascii"))
        if fmt == "ascii":
            for row in cols:
                f.write((" ".join(repr(float(v)) for v in row) + "\n").encode("ascii"))
        else:
            f.write(np.ascontiguousarray(cols.astype("<f4" if fmt == "binary_little_endian" else ">f4")).tobytes())

