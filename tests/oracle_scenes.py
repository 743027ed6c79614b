"""Small hand-built scenes for oracle pins (CPU only)."""
from __future__ import annotations

import numpy as np

import gs_inputs
from gs_inputs import Camera, Scene


def identity_camera(width: int, height: int, f: float, z0: float = 0.0) -> Camera:
    """Camera at (0, 0, -z0) looking down +z with axes aligned to the world."""
    return Camera(np.eye(3, dtype=np.float32), np.array([0.0, 0.0, z0], dtype=np.float32),
                  float(np.float32(f)), float(np.float32(f)), width / 2.0, height / 2.0, width, height)


def scene_from(means, scales, quats, opacity, dc_rgb=None, sh=None, degree=0) -> Scene:
    means = np.asarray(means, dtype=np.float32).reshape(-1, 3).T.copy()
    n = means.shape[1]
    scales = np.asarray(scales, dtype=np.float32).reshape(n, 3).T.copy()
    quats = np.asarray(quats, dtype=np.float32).reshape(n, 4).T.copy()
    opacity = np.asarray(opacity, dtype=np.float32).reshape(n).copy()
    if sh is None:
        sh = np.zeros((16, 3, n), dtype=np.float32)
        if dc_rgb is not None:
            y00 = 0.5 / np.sqrt(np.pi)
            sh[0] = ((np.asarray(dc_rgb, dtype=np.float64).reshape(n, 3) - 0.5) / y00).T
    return Scene(means, scales, quats, opacity, np.asarray(sh, dtype=np.float32), degree)


def random_small_scene(seed: int, n: int = 12, spread: float = 0.6, scale_lo: float = 0.08,
                       scale_hi: float = 0.3, degree: int = 3) -> Scene:
    g = gs_inputs.rng(seed)
    means = g.uniform(-spread, spread, size=(3, n)).astype(np.float32)
    scales = g.uniform(scale_lo, scale_hi, size=(3, n)).astype(np.float32)
    q = g.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    opacity = g.uniform(0.2, 0.9, size=n).astype(np.float32)
    sh = np.zeros((16, 3, n), dtype=np.float32)
    sh[0] = g.normal(0.6, 0.3, size=(3, n))
    sh[1:] = g.normal(0.0, 0.15, size=(15, 3, n))
    return Scene(means, scales, q.astype(np.float32), opacity, sh, degree)
