"""Pins for the oracle's integer binning: numpy emission + lexsort (library
sort), ranges by counting, multiplicity of each record."""
import numpy as np
import pytest

import gs_inputs
import oracle


def _random_rects(seed, n_views, n, tiles_x, tiles_y):
    g = gs_inputs.rng(seed)
    rects = np.zeros((n_views * n, 4), dtype=np.int32)
    for r in range(n_views * n):
        v = r // n
        if g.uniform() < 0.15:
            rects[r] = (1, 0, 1, 0)
            continue
        x0 = g.integers(0, tiles_x[v])
        y0 = g.integers(0, tiles_y[v])
        rects[r] = (x0, min(tiles_x[v] - 1, x0 + g.integers(0, 3)), y0, min(tiles_y[v] - 1, y0 + g.integers(0, 3)))
    # depths with many exact ties
    zb = (g.integers(0, 40, size=n_views * n) + np.float32(2.0).view(np.uint32)).astype(np.uint32)
    return rects, zb


@pytest.mark.parametrize("seed,n_views", [(0, 1), (1, 3)])
def test_bin_matches_numpy_lexsort(seed, n_views):
    n = 700
    cams = [gs_inputs.look_at((0, 0, 4), (0, 0, 0), w, h) for (w, h) in [(100, 60), (37, 90), (64, 64)][:n_views]]
    tx, ty, base, total = oracle.view_layout(cams)
    rects, zb = _random_rects(seed, n_views, n, tx, ty)
    keys, vals, ranges = oracle.bin(rects, zb, n_views, n, base, tx, total)
    ek, ev = [], []
    for r in range(n_views * n):
        x0, x1, y0, y1 = rects[r]
        v = r // n
        for yy in range(y0, y1 + 1):
            for xx in range(x0, x1 + 1):
                ek.append((int(base[v] + yy * tx[v] + xx) << 32) | int(zb[r]))
                ev.append(r)
    ek = np.array(ek, dtype=np.uint64)
    ev = np.array(ev, dtype=np.uint32)
    perm = np.lexsort((ev, ek))
    assert np.array_equal(keys, ek[perm]) and np.array_equal(vals, ev[perm])
    tile = (keys >> np.uint64(32)).astype(np.int64)
    counts = np.bincount(tile, minlength=total)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    for t in range(total):
        if counts[t]:
            assert tuple(ranges[t]) == (starts[t], starts[t] + counts[t])
        else:
            assert tuple(ranges[t]) == (0, 0)
    mult = np.bincount(vals, minlength=n_views * n)
    ok = (rects[:, 0] <= rects[:, 1]) & (rects[:, 2] <= rects[:, 3])
    expect = np.where(ok, (rects[:, 1] - rects[:, 0] + 1) * (rects[:, 3] - rects[:, 2] + 1), 0)
    assert np.array_equal(mult, expect)


def test_bin_empty():
    keys, vals, ranges = oracle.bin(np.zeros((0, 4), np.int32), np.zeros(0, np.uint32), 1, 0, [0], [4], 12)
    assert len(keys) == 0 and np.all(ranges == 0)
