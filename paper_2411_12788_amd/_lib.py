"""ctypes declarations of the C ABI in include/msplat.h (libmsplat.so).

Argument marshalling only; every computation happens in the HIP library.
Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsplat.so")

GS_MAX_VIEWS = 32
GS_TILE = 16
GS_REC_FLOATS = 16
GS_GRAD2D_FLOATS = 9
GS_OK, GS_ERR_NULL, GS_ERR_SHAPE, GS_ERR_CAMERA, GS_ERR_CAPACITY, GS_ERR_DEVICE, GS_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
GS_DEPTH_MID, GS_DEPTH_CENTER, GS_DEPTH_BLEND = 0, 1, 2
GS_ACCUM_IMPORTANCE, GS_ACCUM_PER_VIEW = 1, 2
GS_THRESHOLD_VALUE, GS_THRESHOLD_MASS = 0, 1
GS_SORT_STATIC_MAX_PAIRS = 1 << 20
GS_SORT_PRESCAN, GS_SORT_LOOKBACK = 0, 1

c_p = ctypes.c_void_p
c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_u32 = ctypes.c_uint32
c_sz = ctypes.c_size_t


class Scene(ctypes.Structure):
    _fields_ = [("means", c_p), ("scales", c_p), ("quats", c_p), ("opacity", c_p), ("sh", c_p), ("n", c_i64),
                ("sh_degree", c_i32)]


class Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("width", c_i32), ("height", c_i32)]


class Opts(ctypes.Structure):
    _fields_ = [("znear", ctypes.c_float), ("lowpass", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("alpha_min", ctypes.c_float), ("t_min", ctypes.c_float), ("jac_clamp", ctypes.c_float),
                ("bg", ctypes.c_float * 3), ("depth_mode", c_i32), ("flags", c_i32)]


class Projected(ctypes.Structure):
    _fields_ = [("rec", c_p), ("bin", c_p), ("tile_cull_log2_alpha", ctypes.c_float)]


class BinStats(ctypes.Structure):
    _fields_ = [("n_isect", c_i64), ("n_visible", c_i64), ("zbits_min", c_u32), ("zbits_max", c_u32),
                ("tiles_total", c_i32), ("depth_bits", c_i32), ("key_bits", c_i32), ("pad", c_i32)]


class FwdOut(ctypes.Structure):
    _fields_ = [("color", c_p), ("depth", c_p), ("imax", c_p), ("t_final", c_p), ("last", c_p), ("n_contrib", c_p),
                ("hit", c_p)]


class Accum(ctypes.Structure):
    _fields_ = [("importance", c_p), ("wmax", c_p), ("area", c_p)]


class Grads(ctypes.Structure):
    _fields_ = [("means", c_p), ("scales", c_p), ("quats", c_p), ("opacity", c_p), ("sh", c_p)]


class SceneOut(ctypes.Structure):
    _fields_ = [("means", c_p), ("scales", c_p), ("quats", c_p), ("opacity", c_p), ("sh", c_p), ("capacity", c_i64)]


P = ctypes.POINTER
_SIGS = {
    "gs_last_error": (ctypes.c_char_p, []),
    "gs_version": (c_i32, []),
    "gs_default_opts": (None, [P(Opts)]),
    "gs_view_layout": (c_i32, [P(Camera), c_i32, c_p, c_p, c_p, c_p, P(c_i32), P(c_i64)]),
    "gs_project": (c_i32, [P(Scene), P(Camera), c_i32, c_p, P(Opts), P(Projected), c_p]),
    "gs_bin_count_workspace_size": (c_sz, [c_i64]),
    "gs_bin_count": (c_i32, [P(Projected), P(Camera), c_i32, c_i64, c_p, P(BinStats), c_p, c_sz, c_p]),
    "gs_bin_sort_workspace_size": (c_sz, [c_i64]),
    "gs_bin_sort": (c_i32, [P(Projected), P(Camera), c_i32, c_i64, c_p, P(BinStats), c_p, c_p, c_p, c_p, c_p, c_sz,
                            c_p]),
    "gs_bin": (c_i32, [P(Projected), P(Camera), c_i32, c_i64, c_p, P(BinStats), c_p, c_p, c_i64, c_p, c_p, c_p, c_sz,
                       c_p, c_sz, c_p]),
    "gs_tile_order_workspace_size": (c_sz, []),
    "gs_tile_order": (c_i32, [c_p, c_i32, c_p, c_p, c_sz, c_p]),
    "gs_emit_keys": (c_i32, [P(Projected), P(Camera), c_i32, c_i64, c_p, c_i32, c_u32, c_p, c_p, c_p]),
    "gs_sort_workspace_size": (c_sz, [c_i64]),
    "gs_sort_pairs": (c_i32, [c_p, c_p, c_i64, c_i32, c_p, c_sz, c_p]),
    "gs_tile_ranges": (c_i32, [c_p, c_i64, c_i32, c_u32, c_i32, c_p, c_p, c_p]),
    "gs_sort_status": (c_i32, [c_p, c_p]),
    "gs_sort_set_spin_limit": (None, [c_u32]),
    "gs_sort_set_algorithm": (c_i32, [c_i32]),
    "gs_bin_count_set_fold_blocks": (c_i64, [c_i64]),
    "gs_sort_pairs_static": (c_i32, [c_p, c_p, c_i64, c_i32, c_p, c_p]),
    "gs_spatial_order_workspace_size": (c_sz, [c_i64]),
    "gs_spatial_order": (c_i32, [c_p, c_i64, c_p, c_p, c_p, c_sz, c_p]),
    "gs_permute": (c_i32, [c_p, c_p, c_i64, c_i64, c_i32, c_p, c_p]),
    "gs_render_forward": (c_i32, [P(Scene), P(Projected), c_p, c_p, c_p, P(Camera), c_i32, P(Opts), P(FwdOut),
                                  P(Accum), c_p]),
    "gs_accumulate_importance": (c_i32, [P(Projected), c_p, c_p, c_p, P(Camera), c_i32, c_i64, P(Opts), P(Accum),
                                         c_p]),
    "gs_render_backward": (c_i32, [P(Scene), P(Projected), c_p, c_p, c_p, P(Camera), c_i32, P(Opts), c_p, c_p, c_p,
                                   c_p, c_p, P(Grads), c_p]),
    "gs_render_backward_pixels": (c_i32, [P(Projected), c_p, c_p, c_p, P(Camera), c_i32, c_i64, P(Opts), c_p, c_p,
                                          c_p, c_p, c_p, c_p]),
    "gs_render_backward_det_workspace_size": (c_sz, [c_i64]),
    "gs_render_backward_pixels_det": (c_i32, [P(Projected), c_p, c_p, c_p, c_p, P(Camera), c_i32, c_i64, c_i64,
                                              P(Opts), c_p, c_p, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "gs_project_backward": (c_i32, [P(Scene), P(Projected), P(Camera), c_i32, P(Opts), c_p, c_p, P(Grads), c_p]),
    "gs_l1_loss_grad": (c_i32, [c_p, c_p, c_i64, c_p, c_p, c_p]),
    "gs_fill_u32": (c_i32, [c_p, c_u32, c_i64, c_p]),
    "gs_select_workspace_size": (c_sz, [c_i32]),
    "gs_visibility": (c_i32, [c_p, c_i32, c_i64, ctypes.c_double, c_i32, c_p, c_p, c_p, c_sz, c_p]),
    "gs_critical": (c_i32, [c_p, c_p, c_i64, ctypes.c_double, c_i32, c_p, c_p, c_p, c_sz, c_p]),
    "gs_blur_split": (c_i32, [c_p, c_i64, ctypes.c_double, c_i32, c_i32, c_p, c_p]),
    "gs_grad_stats": (c_i32, [P(Projected), c_p, P(Camera), c_i32, c_i64, c_p, c_p, c_p]),
    "gs_clone_workspace_size": (c_sz, [c_i64]),
    "gs_clone": (c_i32, [P(Scene), c_p, P(SceneOut), c_p, c_p, c_sz, c_p]),
    "gs_densify_select": (c_i32, [c_p, c_p, c_p, c_i64, ctypes.c_double, ctypes.c_double, c_p, c_p, c_p]),
    "gs_split_workspace_size": (c_sz, [c_i64]),
    "gs_split": (c_i32, [P(Scene), c_p, c_p, ctypes.c_double, P(SceneOut), c_p, c_p, c_sz, c_p]),
    "gs_sample_workspace_size": (c_sz, [c_i64]),
    "gs_sample": (c_i32, [c_p, c_p, c_p, c_i64, c_i64, c_p, c_p, c_p, c_sz, c_p]),
    "gs_depth_points_workspace_size": (c_sz, [c_i64]),
    "gs_depth_points": (c_i32, [c_p, c_p, c_p, c_p, c_p, P(Camera), c_i32, ctypes.c_double, c_i32, c_p, c_p, c_i64,
                                c_p, c_p, c_sz, c_p]),
}

_lib = None


class MsplatError(RuntimeError):
    pass


def lib() -> ctypes.CDLL:
    """The HIP library; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MsplatError(f"{LIB_PATH} is missing: build it with paper_2411_12788_amd/build.py "
                              "(or __graft_entry__.build()); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return list(_SIGS.keys())


def check(status: int, what: str = "") -> None:
    if status != GS_OK:
        msg = lib().gs_last_error()
        raise MsplatError(f"{what} failed with status {status}: {msg.decode() if msg else ''}")
