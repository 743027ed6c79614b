"""The radix sort's error flag reaches the caller (GPU, through the C ABI).

With the look-back passes the sort waits on other workgroups in bounded
loops; a wait that gives up raises a flag in the workspace header instead of
hanging.  These tests force that condition from the host (a spin limit of 0
makes every look-back give up at once, so every kernel still exits normally)
or preset the flag, and check that gs_sort_status reports it and that the
next sort clears it (with either pass algorithm).
"""
import ctypes

import numpy as np
import pytest
import torch

import gs_inputs
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _sort(L, keys, vals, bits, ws):
    return L.lib().gs_sort_pairs(ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()), keys.numel(),
                                 bits, ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)


def _pairs(n, seed):
    g = gs_inputs.rng(seed)
    keys = g.integers(0, 1 << 40, size=n, dtype=np.uint64)
    vals = np.arange(n, dtype=np.uint32)
    return keys, vals


def test_preset_flag_is_reported_and_cleared(gpu_lib):
    from paper_2411_12788_amd import _lib as L
    n = 50_000
    keys, vals = _pairs(n, 5)
    kt = torch.from_numpy(keys.view(np.int64)).cuda()
    vt = torch.from_numpy(vals.view(np.int32)).cuda()
    ws = torch.zeros(L.lib().gs_sort_workspace_size(n), dtype=torch.uint8, device="cuda")
    assert _sort(L, kt, vt, 40, ws) == L.GS_OK
    assert L.lib().gs_sort_status(ctypes.c_void_p(ws.data_ptr()), None) == L.GS_OK
    ws[:4].view(torch.int32).fill_(1)  # as a look-back that gave up would leave it
    assert L.lib().gs_sort_status(ctypes.c_void_p(ws.data_ptr()), None) == L.GS_ERR_DEVICE
    assert b"invalid" in L.lib().gs_last_error()
    assert _sort(L, kt, vt, 40, ws) == L.GS_OK  # the next sort clears the flag
    assert L.lib().gs_sort_status(ctypes.c_void_p(ws.data_ptr()), None) == L.GS_OK


def test_look_back_that_gives_up_is_reported(gpu_lib):
    """Spin limit 0: every workgroup but the first gives up its look-back at
    once; the kernels still exit, the stores stay in bounds, and the caller
    sees the error instead of a silently wrong order."""
    from paper_2411_12788_amd import _lib as L
    n = 200_003  # ~49 tiles of 4096 pairs: many look-backs
    keys, vals = _pairs(n, 6)
    ws = torch.zeros(L.lib().gs_sort_workspace_size(n), dtype=torch.uint8, device="cuda")
    kt = torch.from_numpy(keys.view(np.int64)).cuda()
    vt = torch.from_numpy(vals.view(np.int32)).cuda()
    print(f"spin limit 0, n={n}", flush=True)
    L.lib().gs_sort_set_algorithm(L.GS_SORT_LOOKBACK)
    L.lib().gs_sort_set_spin_limit(0)
    try:
        assert _sort(L, kt, vt, 40, ws) == L.GS_OK  # enqueued fine; the error shows at the status read
        assert L.lib().gs_sort_status(ctypes.c_void_p(ws.data_ptr()), None) == L.GS_ERR_DEVICE
    finally:
        L.lib().gs_sort_set_spin_limit(1 << 22)
        L.lib().gs_sort_set_algorithm(L.GS_SORT_PRESCAN)
    kt = torch.from_numpy(keys.view(np.int64)).cuda()
    vt = torch.from_numpy(vals.view(np.int32)).cuda()
    assert _sort(L, kt, vt, 40, ws) == L.GS_OK
    assert L.lib().gs_sort_status(ctypes.c_void_p(ws.data_ptr()), None) == L.GS_OK
    perm = np.lexsort((vals, keys))
    assert np.array_equal(kt.cpu().numpy().view(np.uint64), keys[perm])
    assert np.array_equal(vt.cpu().numpy().view(np.uint32), vals[perm])


def test_binning_checks_the_flag(gpu_lib):
    """raster.bin reads the flag back after every sort (tests rely on it)."""
    R = H.raster()
    wl = gs_inputs.small_cube(seed=1)
    out = H.run_gpu_forward(wl.scene, wl.cameras, accumulate=False)
    assert out["binned"].stats.n_isect > 0


def test_empty_sorts_leave_a_clear_flag(gpu_lib):
    """No pairs: nothing is sorted, and the flag of a workspace that holds
    stale bytes reads clear (an empty order is valid)."""
    from paper_2411_12788_amd import _lib as L
    R = H.raster()
    ws = torch.full((L.lib().gs_sort_workspace_size(1),), 0xFF, dtype=torch.uint8, device="cuda")
    kt = torch.zeros(1, dtype=torch.int64, device="cuda")
    vt = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert L.lib().gs_sort_pairs(ctypes.c_void_p(kt.data_ptr()), ctypes.c_void_p(vt.data_ptr()), 0, 40,
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), None) == L.GS_OK
    assert L.lib().gs_sort_status(ctypes.c_void_p(ws.data_ptr()), None) == L.GS_OK
    # a view where every Gaussian is culled: zero pairs through gs_bin_sort
    cam = gs_inputs.look_at((0, 0, 4), (0, 0, 0), 37, 23)
    sc = gs_inputs.uniform_cube_scene(500, 3)
    ds = R.DeviceScene.from_numpy(sc)
    proj = R.project(ds, [cam], R.RasterOpts(), torch.zeros(500, dtype=torch.uint8, device="cuda"))
    offsets, st = R.bin_count(proj, [cam], sc.n)
    assert st.n_isect == 0
    bufs = R.BinBuffers()
    bufs.ws = torch.full((L.lib().gs_bin_sort_workspace_size(1),), 0xFF, dtype=torch.uint8, device="cuda")
    R.bin_sort(proj, [cam], sc.n, offsets, st, buffers=bufs)
    R.sort_status(bufs.ws)
