"""Vectorised NumPy restatement of Eq. (1) compositing for tiny inputs.

TEST INFRASTRUCTURE ONLY.  A second, differently shaped formulation of the same
definition used to cross-check the per-pixel loop in oracle.c: instead of a
running transmittance with an early stop, it forms the full [pixels x Gaussians]
alpha matrix, zeroes the skipped entries, takes a cumulative product along
depth order, and keeps the entries whose transmittance *after* them is still at
or above the stop threshold (the cumulative product is non-increasing, so that
set is exactly the prefix before the stop).
"""
from __future__ import annotations

import numpy as np


def composite(u, v, conic, opac, rgb, order, width, height, alpha_max, alpha_min, t_min, bg):
    """u, v, opac: [n]; conic: [n, 3] (a, b, c); rgb: [n, 3]; order: indices in depth order."""
    ys, xs = np.mgrid[0:height, 0:width]
    xc = xs.reshape(-1) + 0.5
    yc = ys.reshape(-1) + 0.5
    o = np.asarray(order)
    dx = xc[:, None] - u[o][None, :]
    dy = yc[:, None] - v[o][None, :]
    a, b, c = conic[o, 0], conic[o, 1], conic[o, 2]
    q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
    alpha = np.minimum(alpha_max, opac[o][None, :] * np.exp(-0.5 * q))
    alpha = np.where(alpha < alpha_min, 0.0, alpha)
    t_after = np.cumprod(1.0 - alpha, axis=1)
    keep = (alpha > 0) & (t_after >= t_min)
    alpha_k = np.where(keep, alpha, 0.0)
    t_after_k = np.cumprod(1.0 - alpha_k, axis=1)
    t_before = np.concatenate([np.ones((alpha.shape[0], 1)), t_after_k[:, :-1]], axis=1)
    w = alpha_k * t_before
    color = w @ rgb[o] + t_after_k[:, -1:] * np.asarray(bg)[None, :] if len(o) else \
        np.tile(np.asarray(bg, dtype=np.float64), (alpha.shape[0], 1))
    t_final = t_after_k[:, -1] if len(o) else np.ones(alpha.shape[0])
    wpos = np.where(w > 0, w, -1.0)
    best = np.where(w.max(axis=1, initial=0) > 0, o[np.argmax(wpos, axis=1)] if len(o) else -1, -1)
    return color, t_final, best, w, o
