"""Pins of the oracle's spatial order (the Morton layout of the GPU library):
octree descent in double precision, the Z-order of known grid cells, numpy's
stable argsort, and the special cases (empty, one point, equal points,
non-finite coordinates, the box's upper face, an extent that overflows)."""
import numpy as np
import pytest

import gs_inputs
import oracle as O

FULL = (1 << 30) - 1


def descent_code(p, lo, hi, levels=10):
    """Code by halving the box: at each level the octant (x, y, z bits, x most
    significant) of the point in the current cell, in double precision."""
    a = np.array(lo, dtype=np.float64)
    b = np.array(hi, dtype=np.float64)
    code = 0
    for _ in range(levels):
        mid = (a + b) / 2
        bits = [int(p[k] >= mid[k]) for k in range(3)]
        for k in range(3):
            if bits[k]:
                a[k] = mid[k]
            else:
                b[k] = mid[k]
        code = (code << 3) | (bits[0] << 2) | (bits[1] << 1) | bits[2]
    return code


def test_codes_match_octree_descent():
    g = gs_inputs.rng(11)
    m = g.uniform(-3.0, 5.0, size=(3, 4000)).astype(np.float32)
    m[1] *= 0.25  # unequal extents per axis
    codes, _ = O.spatial_order(m)
    md = m.astype(np.float64)
    lo, hi = md.min(axis=1), md.max(axis=1)
    u = (md - lo[:, None]) / (hi - lo)[:, None] * 1024.0
    # points whose cell the float32 rounding could move are left out
    clear = np.all(np.abs(u - np.round(u)) > 1e-3, axis=0) & np.all(u < 1023.99, axis=0)
    assert clear.sum() > 3500
    for i in np.flatnonzero(clear)[:1500]:
        assert int(codes[i]) == descent_code(md[:, i], lo, hi), i


def test_codes_of_known_cells():
    # box [0, 1024]^3 fixed by two corners; points at cell centres
    cells = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1], [2, 0, 0], [0, 2, 0],
                      [512, 0, 0], [1023, 1023, 1023], [3, 5, 6]], dtype=np.float64)
    expect = [0, 4, 2, 1, 7, 32, 16, 1 << 29, FULL, 0]
    # (3, 5, 6): bit 0 of (x, y, z) = (1, 1, 0) -> 6; bit 1 = (1, 0, 1) -> 5 << 3;
    # bit 2 = (0, 1, 1) -> 3 << 6
    expect[-1] = 6 | (5 << 3) | (3 << 6)
    pts = np.concatenate([np.zeros((1, 3)), np.full((1, 3), 1024.0), cells + 0.5]).T.astype(np.float32)
    codes, _ = O.spatial_order(pts)
    assert codes[0] == 0 and codes[1] == FULL  # the upper face clamps to cell 1023
    assert [int(c) for c in codes[2:]] == expect


def test_perm_is_stable_argsort():
    g = gs_inputs.rng(12)
    m = g.integers(0, 4, size=(3, 3000)).astype(np.float32)  # many equal codes
    codes, perm = O.spatial_order(m)
    assert np.array_equal(perm, np.argsort(codes, kind="stable"))
    assert np.array_equal(np.sort(perm), np.arange(3000))


def test_special_cases():
    c, p = O.spatial_order(np.zeros((3, 0), np.float32))
    assert c.size == 0 and p.size == 0
    c, p = O.spatial_order(np.array([[1.0], [2.0], [3.0]], np.float32))
    assert c[0] == 0 and p[0] == 0  # zero extent: every cell 0
    c, p = O.spatial_order(np.full((3, 7), 2.5, np.float32))
    assert np.all(c == 0) and np.array_equal(p, np.arange(7))
    # a non-finite coordinate: last, and the box is that of the finite means
    g = gs_inputs.rng(13)
    m = g.uniform(-1, 1, size=(3, 50)).astype(np.float32)
    ref, _ = O.spatial_order(m)
    m2 = np.concatenate([m, np.array([[np.nan, 0, 0], [0, np.inf, 0], [0, 0, -np.inf]], np.float32).T], axis=1)
    c2, p2 = O.spatial_order(m2)
    assert np.array_equal(c2[:50], ref) and np.all(c2[50:] == FULL)
    assert list(p2[-3:]) == [50, 51, 52]
    # extent beyond float32: s = 1024 / inf = 0; the top point's product is
    # inf * 0 (not a number) and takes cell 1023, every other point cell 0
    big = np.array([[-3e38, 3e38, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]], np.float32)
    c, _ = O.spatial_order(big)
    x_cell_1023 = sum(1 << (3 * b + 2) for b in range(10))  # x cell 1023, y and z cells 0
    assert list(c) == [0, x_cell_1023, 0]


def test_order_is_local():
    """Along the order, consecutive Gaussians are much closer than random pairs."""
    sc = gs_inputs.surface_scene(20000, 14)
    _, p = O.spatial_order(sc.means)
    m = sc.means[:, p].astype(np.float64)
    step = np.linalg.norm(np.diff(m, axis=1), axis=0)
    rnd = np.linalg.norm(sc.means[:, 1:] - sc.means[:, :-1], axis=0)
    assert np.median(step) < 0.1 * np.median(rnd)
