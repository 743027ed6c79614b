"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/msplat.h declares, and rejects bad arguments on the host
before any device work."""
import ctypes
import os
import re

import pytest

import gs_inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msplat.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_2411_12788_amd import _lib
    _lib.lib()
    return _lib


def test_library_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 20
    lib = L.lib()
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.exported_names())


def test_default_opts_and_version(L):
    o = L.Opts()
    L.lib().gs_default_opts(ctypes.byref(o))
    assert o.alpha_max == pytest.approx(0.99) and o.alpha_min == pytest.approx(1 / 255)
    assert o.t_min == pytest.approx(1e-4) and o.lowpass == pytest.approx(0.3) and o.znear == pytest.approx(0.2)
    assert o.depth_mode == 0 and o.flags == 0
    assert L.lib().gs_version() >= 100


def test_view_layout_host_only(L):
    from paper_2411_12788_amd import raster as R
    cams = [gs_inputs.look_at((0, 0, 4), (0, 0, 0), w, h) for (w, h) in [(1920, 1080), (37, 23), (16, 16)]]
    lay = R.view_layout(cams)
    assert lay.tiles_x == [120, 3, 1] and lay.tiles_y == [68, 2, 1]
    assert lay.tile_base == [0, 8160, 8166] and lay.tiles_total == 8167
    assert lay.pixel_base == [0, 1920 * 1080, 1920 * 1080 + 37 * 23]


def test_argument_errors_on_host(L):
    from paper_2411_12788_amd import raster as R
    lib = L.lib()
    cams = R.cameras([gs_inputs.look_at((0, 0, 4), (0, 0, 0), 16, 16)])
    o = R.RasterOpts().c()
    out = L.Projected()
    assert lib.gs_project(None, cams, 1, None, ctypes.byref(o), ctypes.byref(out), None) == L.GS_ERR_NULL
    s = L.Scene()
    s.n, s.sh_degree = 4, 3
    assert lib.gs_project(ctypes.byref(s), cams, 1, None, ctypes.byref(o), ctypes.byref(out), None) == L.GS_ERR_NULL
    s.n, s.sh_degree = 0, 5
    assert lib.gs_project(ctypes.byref(s), cams, 1, None, ctypes.byref(o), ctypes.byref(out), None) == L.GS_ERR_SHAPE
    s.sh_degree = 3
    assert lib.gs_project(ctypes.byref(s), cams, 0, None, ctypes.byref(o), ctypes.byref(out), None) == L.GS_ERR_SHAPE
    assert lib.gs_project(ctypes.byref(s), cams, 33, None, ctypes.byref(o), ctypes.byref(out), None) == L.GS_ERR_SHAPE
    cams[0].fy = -1.0
    assert lib.gs_project(ctypes.byref(s), cams, 1, None, ctypes.byref(o), ctypes.byref(out), None) == L.GS_ERR_CAMERA
    cams[0].fy = 10.0
    cams[0].width = 0
    assert lib.gs_project(ctypes.byref(s), cams, 1, None, ctypes.byref(o), ctypes.byref(out), None) == L.GS_ERR_SHAPE
    assert b"size" in lib.gs_last_error()
    assert lib.gs_sort_pairs(None, None, 10, 0, None, 0, None) == L.GS_ERR_SHAPE
    assert lib.gs_sort_pairs(None, None, 0, 8, None, 0, None) == L.GS_OK
    assert lib.gs_fill_u32(None, 0, 0, None) == L.GS_OK
    # the sort's 30-bit per-digit prefixes: 2^30 pairs or more are refused before any launch
    fake = ctypes.c_void_p(0x1000)
    big = 1 << 30
    assert lib.gs_sort_pairs(fake, fake, big, 40, fake, lib.gs_sort_workspace_size(big), None) == L.GS_ERR_CAPACITY
    assert b"2^30" in lib.gs_last_error()
    cams[0].width = 64
    st = L.BinStats()
    st.n_isect, st.tiles_total = big, 4
    proj = L.Projected(fake, fake, 0.0)
    assert lib.gs_bin_sort(ctypes.byref(proj), cams, 1, 10, fake, ctypes.byref(st), fake, fake, fake, None, fake,
                           lib.gs_bin_sort_workspace_size(big), None) == L.GS_ERR_CAPACITY
    assert lib.gs_sort_status(None, None) == L.GS_ERR_NULL
    assert lib.gs_bin_count_workspace_size(10 ** 6) > 0 and lib.gs_bin_sort_workspace_size(10 ** 6) > 12 * 10 ** 6


def test_criteria_argument_errors_on_host(L):
    """Checks that happen before any launch (fake non-NULL pointers are never touched)."""
    lib = L.lib()
    fake = ctypes.c_void_p(0x1000)
    ws = lib.gs_select_workspace_size(2)
    assert ws >= 2 * 4096
    assert lib.gs_visibility(fake, 2, 10, 1.5, 0, fake, fake, fake, ws, None) == L.GS_ERR_SHAPE
    assert lib.gs_visibility(fake, 2, 10, -0.1, 0, fake, fake, fake, ws, None) == L.GS_ERR_SHAPE
    assert lib.gs_visibility(fake, 2, 10, 0.99, 7, fake, fake, fake, ws, None) == L.GS_ERR_UNSUPPORTED
    assert lib.gs_visibility(fake, 2, 10, 0.99, 1, fake, fake, fake, ws - 1, None) == L.GS_ERR_CAPACITY
    assert lib.gs_visibility(fake, 0, 10, 0.99, 1, fake, fake, fake, ws, None) == L.GS_ERR_SHAPE
    assert lib.gs_visibility(fake, 33, 10, 0.99, 1, fake, fake, fake, ws, None) == L.GS_ERR_SHAPE
    assert lib.gs_visibility(None, 2, 10, 0.99, 1, fake, fake, fake, ws, None) == L.GS_ERR_NULL
    assert lib.gs_critical(fake, None, 10, 0.99, 1, fake, fake, fake, ws, None) == L.GS_ERR_NULL
    assert lib.gs_critical(fake, fake, -1, 0.99, 1, fake, fake, fake, ws, None) == L.GS_ERR_SHAPE
    assert lib.gs_blur_split(fake, 10, 2e-4, 0, 10, fake, None) == L.GS_ERR_SHAPE
    assert lib.gs_blur_split(fake, 10, -1.0, 10, 10, fake, None) == L.GS_ERR_SHAPE
    assert lib.gs_blur_split(fake, 0, 2e-4, 10, 10, None, None) == L.GS_OK          # nothing to do
    sc = L.Scene(fake, fake, fake, fake, fake, 100, 3)
    out = L.SceneOut(fake, fake, fake, fake, fake, 99)
    cw = lib.gs_clone_workspace_size(100)
    assert lib.gs_clone(ctypes.byref(sc), fake, ctypes.byref(out), fake, fake, cw, None) == L.GS_ERR_CAPACITY
    out.capacity = 200
    assert lib.gs_clone(ctypes.byref(sc), fake, ctypes.byref(out), None, fake, cw, None) == L.GS_ERR_NULL
    assert lib.gs_clone(ctypes.byref(sc), fake, ctypes.byref(out), fake, fake, 0, None) == L.GS_ERR_CAPACITY
    assert lib.gs_clone(ctypes.byref(sc), fake, None, fake, fake, cw, None) == L.GS_ERR_NULL
    # split and the density-control selection
    out.capacity = 99
    sw = lib.gs_split_workspace_size(100)
    assert lib.gs_split(ctypes.byref(sc), fake, fake, 1.6, ctypes.byref(out), fake, fake, sw, None) == L.GS_ERR_CAPACITY
    out.capacity = 200
    assert lib.gs_split(ctypes.byref(sc), fake, fake, 0.0, ctypes.byref(out), fake, fake, sw, None) == L.GS_ERR_SHAPE
    assert lib.gs_split(ctypes.byref(sc), fake, None, 1.6, ctypes.byref(out), fake, fake, sw, None) == L.GS_ERR_NULL
    assert lib.gs_split(ctypes.byref(sc), fake, fake, 1.6, ctypes.byref(out), fake, fake, 0, None) == L.GS_ERR_CAPACITY
    assert lib.gs_densify_select(fake, fake, fake, -1, 1e-4, 0.1, fake, fake, None) == L.GS_ERR_SHAPE
    assert lib.gs_densify_select(fake, fake, fake, 10, 1e-4, 0.1, None, None, None) == L.GS_ERR_NULL
    assert lib.gs_densify_select(None, fake, fake, 10, 1e-4, 0.1, fake, None, None) == L.GS_ERR_NULL
    assert lib.gs_densify_select(None, None, None, 0, 1e-4, 0.1, None, None, None) == L.GS_OK  # nothing to do


def test_static_sort_capacity_on_host(L):
    """Sizes beyond the allocation-free sort's fixed scratch are rejected
    before any device work."""
    lib = L.lib()
    fake = ctypes.c_void_p(0x1000)
    assert lib.gs_sort_pairs_static(fake, fake, L.GS_SORT_STATIC_MAX_PAIRS + 1, 40, None, None) == L.GS_ERR_CAPACITY
    assert lib.gs_sort_pairs_static(fake, fake, 10, 0, None, None) == L.GS_ERR_SHAPE
    assert lib.gs_sort_pairs_static(None, None, 10, 40, None, None) == L.GS_ERR_NULL


def test_sort_algorithm_switch_on_host(L):
    lib = L.lib()
    assert lib.gs_sort_set_algorithm(7) == L.GS_ERR_UNSUPPORTED
    assert lib.gs_sort_set_algorithm(L.GS_SORT_LOOKBACK) == L.GS_OK
    assert lib.gs_sort_set_algorithm(L.GS_SORT_PRESCAN) == L.GS_OK


def test_count_fold_switch_on_host(L):
    lib = L.lib()
    assert lib.gs_bin_count_set_fold_blocks(0) == 4096  # the default
    assert lib.gs_bin_count_set_fold_blocks(-1) == 0
    assert lib.gs_bin_count_set_fold_blocks(-1) == 4096  # restored


def test_fused_binning_argument_errors_on_host(L):
    """gs_bin refuses a negative capacity before anything runs, and passes the
    pair count's argument errors through."""
    from paper_2411_12788_amd import raster as R
    lib = L.lib()
    cams = R.cameras([gs_inputs.look_at((0, 0, 4), (0, 0, 0), 16, 16)])
    fake = ctypes.c_void_p(0x1000)
    st = L.BinStats()
    proj = L.Projected(fake, fake, 0.0)
    assert lib.gs_bin(ctypes.byref(proj), cams, 1, 10, fake, ctypes.byref(st), None, fake, -1, fake, None, fake,
                      1 << 20, fake, 1 << 20, None) == L.GS_ERR_SHAPE
    assert lib.gs_bin(None, cams, 1, 10, fake, ctypes.byref(st), None, fake, 10, fake, None, fake, 1 << 20, fake,
                      1 << 20, None) == L.GS_ERR_NULL
    assert lib.gs_bin(ctypes.byref(proj), cams, 1, 10, fake, None, None, fake, 10, fake, None, fake, 1 << 20, fake,
                      1 << 20, None) == L.GS_ERR_NULL
