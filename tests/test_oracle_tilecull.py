"""Pins of oracle.tile_alpha_max, the per-tile alpha maximum used to check the
renderer's tile culling at emission (Eq. (1): alpha = opacity * G2D)."""
import math

import numpy as np
import pytest

import oracle
from oracle import F


def _row(u, v, sigma_x, sigma_y, o, box):
    P = np.zeros(oracle.STRIDE)
    P[F["U"]], P[F["V"]] = u, v
    P[F["CA"]], P[F["CB"]], P[F["CC"]] = 1.0 / sigma_x ** 2, 0.0, 1.0 / sigma_y ** 2
    P[F["OPAC"]] = o
    P[F["XLO"]], P[F["XHI"]], P[F["YLO"]], P[F["YHI"]] = box
    return P


@pytest.mark.parametrize("u,v", [(3.2, 40.7), (20.0, 20.0), (70.3, 5.5), (15.5, 17.5)])
def test_axis_aligned_closed_form(u, v):
    # the maximum sits at the pixel centre nearest to the mean in each axis
    sx, sy, o = 2.5, 4.0, 0.7
    box = (0, 99, 0, 99)
    P = _row(u, v, sx, sy, o, box)
    for tx, ty in [(0, 0), (1, 1), (4, 0), (0, 2)]:
        cx = min(max(math.floor(u), tx * 16), tx * 16 + 15) + 0.5
        cy = min(max(math.floor(v), ty * 16), ty * 16 + 15) + 0.5
        want = o * math.exp(-0.5 * (((cx - u) / sx) ** 2 + ((cy - v) / sy) ** 2))
        assert oracle.tile_alpha_max(P, tx, ty) == pytest.approx(want, rel=1e-12)


def test_box_limits_the_pixels():
    P = _row(8.0, 8.0, 3.0, 3.0, 0.5, (20, 40, 0, 15))  # box starts right of the mean
    got = oracle.tile_alpha_max(P, 1, 0)
    want = 0.5 * math.exp(-0.5 * ((20.5 - 8.0) / 3.0) ** 2 - 0.5 * ((8.5 - 8.0) / 3.0) ** 2)
    assert got == pytest.approx(want, rel=1e-12)
    assert oracle.tile_alpha_max(P, 0, 0) == 0.0  # tile 0 holds no pixel of the box
