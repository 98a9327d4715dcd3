"""Hand-built tiny scenes and cameras for closed-form and edge-case tests.

Input construction only (no rasterizer arithmetic): colours are set through
the degree-0 SH coefficient so that 0.5 + Y00 * k equals the wanted value.
"""
import math

import numpy as np

from paper_2605_08699_amd.synth import Intrinsics, Pose, Scene

Y00 = 0.5 / math.sqrt(math.pi)
F32 = np.float32


def dc_for(color):
    return (np.asarray(color, np.float64) - 0.5) / Y00


def make_scene(means, log_scales=None, quats=None, logits=None, colors=None, sh_degree=0):
    means = np.asarray(means, np.float64).reshape(-1, 3)
    n = means.shape[0]
    ls = np.full((n, 3), math.log(0.05)) if log_scales is None else np.asarray(log_scales, np.float64).reshape(n, 3)
    q = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)) if quats is None else np.asarray(quats, np.float64).reshape(n, 4)
    lo = np.zeros(n) if logits is None else np.asarray(logits, np.float64).reshape(n)
    cols = np.full((n, 3), 0.5) if colors is None else np.asarray(colors, np.float64).reshape(n, 3)
    sh = np.zeros((n, 16, 3))
    sh[:, 0, :] = dc_for(cols)
    return Scene(means.astype(F32), ls.astype(F32), q.astype(F32), lo.astype(F32), sh.astype(F32), sh_degree)


def eye_pose(t=(0.0, 0.0, 0.0)):
    return Pose(np.eye(3, dtype=F32), np.asarray(t, F32))


def intr(f, cx, cy):
    return Intrinsics(float(f), float(f), float(cx), float(cy))


def random_tiny_scene(rng, n=48, extent=1.0, depth=(2.0, 4.0)):
    """Small random scene in front of an identity camera at the origin, with a
    few Gaussians behind the camera, off-screen, straddling tile edges and
    sharing depths."""
    means = np.column_stack([rng.uniform(-extent, extent, n), rng.uniform(-extent, extent, n),
                             rng.uniform(depth[0], depth[1], n)])
    means[0, 2] = -1.0                       # behind the camera
    means[1] = [40.0, 0.0, 3.0]              # far off-screen
    means[2, 2] = 0.1                        # in front of the near plane
    means[4] = means[3]                      # identical position: equal depth key
    means[6, 2] = means[5, 2]                # equal depth, different place
    ls = rng.normal(-2.5, 0.5, (n, 3))
    q = rng.normal(size=(n, 4))
    logits = rng.normal(0.0, 1.5, n)
    cols = rng.uniform(0.0, 1.0, (n, 3))
    s = make_scene(means, ls, q, logits, cols, sh_degree=3)
    s.sh[:, 1:, :] = rng.normal(0.0, 0.05, (n, 15, 3)).astype(F32)
    return s
