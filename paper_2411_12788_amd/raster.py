"""Thin Python layer over the C ABI: torch tensors in, torch tensors out.

PyTorch only allocates device memory and supplies the stream; every step of
the rasterizer runs in libmsplat.so.  Function names follow the C entry points.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


@dataclasses.dataclass
class RasterOpts:
    znear: float = 0.2
    lowpass: float = 0.3
    alpha_max: float = 0.99
    alpha_min: float = 1.0 / 255.0
    t_min: float = 1e-4
    jac_clamp: float = 1.3
    bg: Sequence[float] = (0.0, 0.0, 0.0)
    depth_mode: int = L.GS_DEPTH_MID
    flags: int = 0
    tile_cull: bool = False  # bin only the tiles a record's alpha >= alpha_min region can reach

    def c(self, flags: Optional[int] = None) -> L.Opts:
        o = L.Opts()
        o.znear, o.lowpass, o.alpha_max, o.alpha_min = self.znear, self.lowpass, self.alpha_max, self.alpha_min
        o.t_min, o.jac_clamp = self.t_min, self.jac_clamp
        for k in range(3):
            o.bg[k] = float(self.bg[k])
        o.depth_mode = int(self.depth_mode)
        o.flags = int(self.flags if flags is None else flags)
        return o


@dataclasses.dataclass
class DeviceScene:
    """Gaussian parameters as device tensors in the library's SoA layout."""
    means: torch.Tensor    # [3, n]
    scales: torch.Tensor   # [3, n]
    quats: torch.Tensor    # [4, n]
    opacity: torch.Tensor  # [n]
    sh: torch.Tensor       # [16, 3, n]
    sh_degree: int = 3

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])

    @staticmethod
    def from_numpy(scene, device="cuda") -> "DeviceScene":
        def t(a):
            return torch.from_numpy(a).to(device=device, dtype=torch.float32).contiguous()
        return DeviceScene(t(scene.means), t(scene.scales), t(scene.quats), t(scene.opacity), t(scene.sh),
                           int(scene.sh_degree))

    def c(self) -> L.Scene:
        for a in (self.means, self.scales, self.quats, self.opacity, self.sh):
            assert a.is_contiguous() and a.dtype == torch.float32
        s = L.Scene()
        s.means, s.scales, s.quats = _ptr(self.means), _ptr(self.scales), _ptr(self.quats)
        s.opacity, s.sh = _ptr(self.opacity), _ptr(self.sh)
        s.n, s.sh_degree = self.n, int(self.sh_degree)
        return s

    def nbytes(self) -> int:
        return sum(a.numel() * 4 for a in (self.means, self.scales, self.quats, self.opacity, self.sh))

    def in_spatial_order(self, stream=None) -> Tuple["DeviceScene", torch.Tensor]:
        """(the scene along the Morton curve of its means, the permutation):
        the layout the compositing kernels read fastest (see spatial_order)."""
        perm = spatial_order(self.means, stream)
        return self.permuted(perm, stream), perm

    def permuted(self, perm: torch.Tensor, stream=None) -> "DeviceScene":
        """The same Gaussians in the order `perm` gives (Gaussian i of the
        result is Gaussian perm[i] of this scene)."""
        return DeviceScene(permute(self.means, perm, stream), permute(self.scales, perm, stream),
                           permute(self.quats, perm, stream), permute(self.opacity, perm, stream),
                           permute(self.sh, perm, stream), self.sh_degree)


def cameras(cams) -> "ctypes.Array[L.Camera]":
    arr = (L.Camera * len(cams))()
    for k, c in enumerate(cams):
        Rm = np.asarray(c.R, dtype=np.float32).reshape(9)
        tv = np.asarray(c.t, dtype=np.float32).reshape(3)
        for i in range(9):
            arr[k].R[i] = float(Rm[i])
        for i in range(3):
            arr[k].t[i] = float(tv[i])
        arr[k].fx, arr[k].fy, arr[k].cx, arr[k].cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        arr[k].width, arr[k].height = int(c.width), int(c.height)
    return arr


@dataclasses.dataclass
class Layout:
    tiles_x: List[int]
    tiles_y: List[int]
    tile_base: List[int]
    pixel_base: List[int]
    tiles_total: int
    pixels_total: int


_LAYOUTS: Dict[tuple, Layout] = {}


def view_layout(cams) -> Layout:
    """Per-view tile and pixel bases of a multi-view launch (from the library).
    It depends only on the views' sizes and is memoised on them: every
    render call asks for it, and building the camera array costs more than
    the lookup (the returned object is shared; do not modify it)."""
    key = tuple((int(c.width), int(c.height)) for c in cams)
    hit = _LAYOUTS.get(key)
    if hit is not None:
        return hit
    V = len(cams)
    ca = cameras(cams)
    tx, ty, tb = (ctypes.c_int32 * V)(), (ctypes.c_int32 * V)(), (ctypes.c_int32 * V)()
    pb = (ctypes.c_int64 * V)()
    tt, pt = ctypes.c_int32(), ctypes.c_int64()
    L.check(L.lib().gs_view_layout(ca, V, tx, ty, tb, pb, ctypes.byref(tt), ctypes.byref(pt)), "gs_view_layout")
    lay = Layout(list(tx), list(ty), list(tb), list(pb), tt.value, pt.value)
    if len(_LAYOUTS) < 1024:
        _LAYOUTS[key] = lay
    return lay


@dataclasses.dataclass
class Projected:
    rec: torch.Tensor  # [V*n, 16] float32
    bin: torch.Tensor  # [V*n, 4] int32
    tile_cull_log2_alpha: float = 0.0  # < 0: binning keeps only reachable tiles

    def c(self) -> L.Projected:
        p = L.Projected()
        p.rec, p.bin = _ptr(self.rec), _ptr(self.bin)
        p.tile_cull_log2_alpha = float(self.tile_cull_log2_alpha)
        return p


class StepBuffers:
    """Reusable device buffers of one stream's projection records, pair count
    and sorted lists, grown when a call needs more (a serving slot or a
    training loop then stops allocating after its first few calls)."""

    def __init__(self):
        self.store: Dict[str, torch.Tensor] = {}
        self.bins = BinBuffers()

    def take(self, name, count, dtype, dev, shape_tail=()):
        per = int(np.prod(shape_tail)) if shape_tail else 1
        base = self.store.get(name)
        if base is None or base.numel() < count * per or base.dtype != dtype:
            base = torch.empty(((count + count // 8) * per,), device=dev, dtype=dtype)
            self.store[name] = base
        return base[: count * per].view((count,) + tuple(shape_tail))


def project(scene: DeviceScene, cams, opts: RasterOpts, cull_mask: Optional[torch.Tensor] = None,
            stream=None, buffers: Optional[StepBuffers] = None) -> Projected:
    V, n = len(cams), scene.n
    dev = scene.opacity.device
    m = max(V * n, 1)
    if buffers is not None:
        rec = buffers.take("rec", m, torch.float32, dev, (L.GS_REC_FLOATS,))
        binr = buffers.take("bin", m, torch.int32, dev, (4,))
    else:
        rec = torch.empty((m, L.GS_REC_FLOATS), device=dev, dtype=torch.float32)
        binr = torch.empty((m, 4), device=dev, dtype=torch.int32)
    out = Projected(rec, binr, float(np.log2(opts.alpha_min)) if opts.tile_cull else 0.0)
    L.check(L.lib().gs_project(ctypes.byref(scene.c()), cameras(cams), V, _ptr(cull_mask), ctypes.byref(opts.c()),
                               ctypes.byref(out.c()), _stream(stream)), "gs_project")
    return out


@dataclasses.dataclass
class Binned:
    vals: torch.Tensor     # [n_isect] uint32 as int32
    ranges: torch.Tensor   # [tiles_total, 2] uint32 as int32
    keys: Optional[torch.Tensor]
    stats: L.BinStats
    offsets: torch.Tensor
    order: Optional[torch.Tensor] = None  # [tiles_total] tile processing order (longest lists first)


def bin_count(proj: Projected, cams, n: int, stream=None, buffers: Optional[StepBuffers] = None):
    V = len(cams)
    dev = proj.rec.device
    need = L.lib().gs_bin_count_workspace_size(V * n)
    if buffers is not None:
        offsets = buffers.take("offsets", max(V * n, 1), torch.int32, dev)
        ws = buffers.take("count_ws", max(need, 1), torch.uint8, dev)
    else:
        offsets = torch.empty(max(V * n, 1), device=dev, dtype=torch.int32)
        ws = torch.empty(need, device=dev, dtype=torch.uint8)
    st = L.BinStats()
    L.check(L.lib().gs_bin_count(ctypes.byref(proj.c()), cameras(cams), V, n, _ptr(offsets), ctypes.byref(st),
                                 _ptr(ws), ws.numel(), _stream(stream)), "gs_bin_count")
    return offsets, st


class BinBuffers:
    """Reusable device buffers of bin_sort (grown when a call needs more), so
    a training loop does not allocate between the pair count and the sort."""

    def __init__(self):
        self.vals = self.keys = self.ranges = self.order = self.ws = None

    @staticmethod
    def _fit(t, count, dtype, dev):
        if t is None or t.numel() < count:
            return torch.empty(count + count // 8, device=dev, dtype=dtype)
        return t

    def get(self, ni, tiles, want_keys, dev):
        self.vals = self._fit(self.vals, max(ni, 1), torch.int32, dev)
        if want_keys:
            self.keys = self._fit(self.keys, max(ni, 1), torch.int64, dev)
        self.ranges = self._fit(self.ranges, 2 * max(tiles, 1), torch.int32, dev)
        self.order = self._fit(self.order, max(tiles, 1), torch.int32, dev)
        self.ws = self._fit(self.ws, max(L.lib().gs_bin_sort_workspace_size(ni), 1), torch.uint8, dev)
        return self.vals, (self.keys if want_keys else None), self.ranges, self.order, self.ws


def bin_sort(proj: Projected, cams, n: int, offsets: torch.Tensor, st: L.BinStats, want_keys: bool = False,
             stream=None, buffers: Optional[BinBuffers] = None) -> Binned:
    """With `buffers` the pair lists live in (and are overwritten on the next
    call with) those reusable buffers."""
    V = len(cams)
    dev = proj.rec.device
    ni = int(st.n_isect)
    tiles = int(st.tiles_total)
    if buffers is None:
        buffers = BinBuffers()
    vals, keys, ranges, order, ws = buffers.get(ni, tiles, want_keys, dev)
    L.check(L.lib().gs_bin_sort(ctypes.byref(proj.c()), cameras(cams), V, n, _ptr(offsets), ctypes.byref(st),
                                _ptr(keys), _ptr(vals), _ptr(ranges), _ptr(order), _ptr(ws), ws.numel(),
                                _stream(stream)), "gs_bin_sort")
    return Binned(vals[:ni], ranges[: 2 * tiles].view(tiles, 2), None if keys is None else keys[:ni], st, offsets,
                  order[:tiles])


def tiles_total(cams) -> int:
    return sum(((int(c.width) + L.GS_TILE - 1) // L.GS_TILE) * ((int(c.height) + L.GS_TILE - 1) // L.GS_TILE)
               for c in cams)


def bin_step(proj: Projected, cams, n: int, buffers: StepBuffers, want_keys: bool = False, stream=None,
             on_count=None) -> Binned:
    """Pair count, emission, sort, ranges and tile order in one library call
    (gs_bin) into the reusable buffers, so nothing runs on the host between
    the pair count's read-back and the sort's launch; when the pairs outgrow
    the buffers they grow and the sort runs as a second call.  on_count(stats),
    if given, runs once the pair count is known and before any buffer grows
    (a caller that accounts for device memory adjusts its reservation there)."""
    V = len(cams)
    dev = proj.rec.device
    lib = L.lib()
    offsets = buffers.take("offsets", max(V * n, 1), torch.int32, dev)
    cws = buffers.take("count_ws", max(lib.gs_bin_count_workspace_size(V * n), 1), torch.uint8, dev)
    bb = buffers.bins
    tiles = tiles_total(cams)
    bb.ranges = bb._fit(bb.ranges, 2 * max(tiles, 1), torch.int32, dev)
    bb.order = bb._fit(bb.order, max(tiles, 1), torch.int32, dev)
    cap = 0 if bb.vals is None else bb.vals.numel()
    if want_keys:
        cap = min(cap, 0 if bb.keys is None else bb.keys.numel())
    ws_bytes = 0 if bb.ws is None else bb.ws.numel()
    st = L.BinStats()
    pc = proj.c()
    cc = cameras(cams)
    sp = _stream(stream)
    rc = lib.gs_bin(ctypes.byref(pc), cc, V, n, _ptr(offsets), ctypes.byref(st), _ptr(bb.keys if want_keys else None),
                    _ptr(bb.vals), cap, _ptr(bb.ranges), _ptr(bb.order), _ptr(cws), cws.numel(), _ptr(bb.ws), ws_bytes,
                    sp)
    ni = int(st.n_isect)
    grow = rc == L.GS_ERR_CAPACITY and 0 <= ni < (1 << 30) and (ni > cap or
                                                                ws_bytes < lib.gs_bin_sort_workspace_size(ni))
    if on_count is not None and (rc == L.GS_OK or grow):
        on_count(st)
    if grow:
        vals, keys, ranges, order, ws = bb.get(ni, tiles, want_keys, dev)
        L.check(lib.gs_bin_sort(ctypes.byref(pc), cc, V, n, _ptr(offsets), ctypes.byref(st), _ptr(keys), _ptr(vals),
                                _ptr(ranges), _ptr(order), _ptr(ws), ws.numel(), sp), "gs_bin_sort")
    else:
        L.check(rc, "gs_bin")
    return Binned(bb.vals[:ni], bb.ranges[: 2 * tiles].view(tiles, 2), bb.keys[:ni] if want_keys else None, st,
                  offsets, bb.order[:tiles])


def sort_status(ws: torch.Tensor, stream=None) -> None:
    """Raises if the last sort on workspace `ws` raised its error flag (synchronises)."""
    L.check(L.lib().gs_sort_status(_ptr(ws), _stream(stream)), "gs_sort_status")


def bin(proj: Projected, cams, n: int, want_keys: bool = False, stream=None, check: bool = True) -> Binned:
    """Pair count, key emission, sort and ranges; with `check` the sort's
    status flag is read back (one synchronisation)."""
    offsets, st = bin_count(proj, cams, n, stream)
    buffers = BinBuffers()
    out = bin_sort(proj, cams, n, offsets, st, want_keys, stream, buffers)
    if check:
        sort_status(buffers.ws, stream)
    return out


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor, key_bits: int, stream=None, check: bool = True) -> None:
    n = keys.numel()
    ws = torch.empty(max(L.lib().gs_sort_workspace_size(n), 1), device=keys.device, dtype=torch.uint8)
    L.check(L.lib().gs_sort_pairs(_ptr(keys), _ptr(vals), n, key_bits, _ptr(ws), ws.numel(), _stream(stream)),
            "gs_sort_pairs")
    if check and n > 0:
        sort_status(ws, stream)


def spatial_order(means: torch.Tensor, stream=None, codes: bool = False):
    """Permutation [n] (int32 holding the library's u32) that stores the
    Gaussians along the Morton curve of their means [3, n]; with `codes` also
    the 30-bit code of each Gaussian.  A memory layout, not a step of the
    method: every result is the same up to the permutation."""
    assert means.dim() == 2 and means.shape[0] == 3 and means.is_contiguous() and means.dtype == torch.float32
    n = int(means.shape[1])
    perm = torch.empty(n, device=means.device, dtype=torch.int32)
    c = torch.empty(n, device=means.device, dtype=torch.int32) if codes else None
    ws = torch.empty(max(L.lib().gs_spatial_order_workspace_size(n), 1), device=means.device, dtype=torch.uint8)
    L.check(L.lib().gs_spatial_order(_ptr(means), n, _ptr(perm), _ptr(c), _ptr(ws), ws.numel(), _stream(stream)),
            "gs_spatial_order")
    return (perm, c) if codes else perm


def permute(t: torch.Tensor, perm: torch.Tensor, stream=None) -> torch.Tensor:
    """New tensor r with r[..., i] = t[..., perm[i]]: the planes of a
    contiguous per-Gaussian array (last dimension n) moved into the order perm
    gives; entries of perm outside [0, n) give zeros."""
    assert t.is_contiguous() and perm.is_contiguous() and perm.dtype == torch.int32
    n = int(t.shape[-1]) if t.dim() > 0 else 0
    assert perm.numel() == n
    out = torch.empty_like(t)
    planes = t.numel() // n if n > 0 else 0
    L.check(L.lib().gs_permute(_ptr(t), _ptr(out), planes, n, t.element_size(), _ptr(perm), _stream(stream)),
            "gs_permute")
    return out


@dataclasses.dataclass
class Frame:
    color: torch.Tensor     # [3, P]
    depth: torch.Tensor     # [P]
    imax: torch.Tensor      # [P]
    t_final: torch.Tensor   # [P]
    last: torch.Tensor      # [P]
    n_contrib: Optional[torch.Tensor]
    hit: Optional[torch.Tensor]


def alloc_accum(n: int, V: int = 1, per_view: bool = False, device="cuda"):
    m = n * (V if per_view else 1)
    return dict(importance=torch.zeros(max(m, 1), device=device), wmax=torch.zeros(max(m, 1), device=device),
                area=torch.zeros(max(m, 1), device=device, dtype=torch.int32))


def _accum_c(acc: Optional[Dict[str, torch.Tensor]]):
    a = L.Accum()
    if acc is not None:
        a.importance, a.wmax, a.area = _ptr(acc.get("importance")), _ptr(acc.get("wmax")), _ptr(acc.get("area"))
    return a


def render_forward(scene: DeviceScene, proj: Projected, binned: Binned, cams, opts: RasterOpts,
                   accum: Optional[Dict[str, torch.Tensor]] = None, extras: bool = True, stream=None,
                   out: Optional[Frame] = None) -> Frame:
    lay_P = view_layout(cams).pixels_total
    dev = proj.rec.device
    if out is None:
        out = Frame(torch.empty((3, lay_P), device=dev), torch.empty(lay_P, device=dev),
                    torch.empty(lay_P, device=dev, dtype=torch.int32), torch.empty(lay_P, device=dev),
                    torch.empty(lay_P, device=dev, dtype=torch.int32),
                    torch.empty(lay_P, device=dev, dtype=torch.int32) if extras else None,
                    torch.empty(lay_P, device=dev, dtype=torch.uint8) if extras else None)
    fo = L.FwdOut()
    fo.color, fo.depth, fo.imax, fo.t_final = _ptr(out.color), _ptr(out.depth), _ptr(out.imax), _ptr(out.t_final)
    fo.last, fo.n_contrib, fo.hit = _ptr(out.last), _ptr(out.n_contrib), _ptr(out.hit)
    flags = opts.flags | (L.GS_ACCUM_IMPORTANCE if accum is not None else 0)
    a = _accum_c(accum)
    L.check(L.lib().gs_render_forward(ctypes.byref(scene.c()), ctypes.byref(proj.c()), _ptr(binned.vals),
                                      _ptr(binned.ranges), _ptr(binned.order), cameras(cams), len(cams),
                                      ctypes.byref(opts.c(flags)),
                                      ctypes.byref(fo), ctypes.byref(a) if accum is not None else None,
                                      _stream(stream)), "gs_render_forward")
    return out


def accumulate_importance(proj: Projected, binned: Binned, cams, n: int, opts: RasterOpts,
                          accum: Dict[str, torch.Tensor], stream=None) -> None:
    a = _accum_c(accum)
    L.check(L.lib().gs_accumulate_importance(ctypes.byref(proj.c()), _ptr(binned.vals), _ptr(binned.ranges),
                                             _ptr(binned.order), cameras(cams), len(cams), n, ctypes.byref(opts.c()),
                                             ctypes.byref(a),
                                             _stream(stream)), "gs_accumulate_importance")


def alloc_grads(n: int, device="cuda") -> Dict[str, torch.Tensor]:
    return dict(means=torch.empty((3, n), device=device), scales=torch.empty((3, n), device=device),
                quats=torch.empty((4, n), device=device), opacity=torch.empty(n, device=device),
                sh=torch.empty((16, 3, n), device=device))


def _grads_c(g):
    c = L.Grads()
    c.means, c.scales, c.quats, c.opacity, c.sh = (_ptr(g["means"]), _ptr(g["scales"]), _ptr(g["quats"]),
                                                   _ptr(g["opacity"]), _ptr(g["sh"]))
    return c


def render_backward(scene: DeviceScene, proj: Projected, binned: Binned, cams, opts: RasterOpts, frame: Frame,
                    dl_dcolor: torch.Tensor, active: Optional[torch.Tensor] = None,
                    grads: Optional[Dict[str, torch.Tensor]] = None, grad2d: Optional[torch.Tensor] = None,
                    stream=None, deterministic: bool = False):
    """Pixel backward then projection backward.  With `deterministic` the
    pixel stage uses the ordered reduction (gradients bitwise the same from
    run to run); the projection backward is per Gaussian and always is."""
    V, n = len(cams), scene.n
    dev = proj.rec.device
    if grads is None:
        grads = alloc_grads(max(n, 1), dev)
    if grad2d is None:
        grad2d = torch.empty((max(V * n, 1), L.GS_GRAD2D_FLOATS), device=dev)
    if deterministic:
        fill_u32(grad2d, 0, stream)
        render_backward_pixels(proj, binned, cams, n, opts, frame, dl_dcolor, active, grad2d, stream,
                               deterministic=True)
        L.check(L.lib().gs_project_backward(ctypes.byref(scene.c()), ctypes.byref(proj.c()), cameras(cams), V,
                                            ctypes.byref(opts.c()), _ptr(grad2d), _ptr(active),
                                            ctypes.byref(_grads_c(grads)), _stream(stream)), "gs_project_backward")
        return grads, grad2d
    L.check(L.lib().gs_render_backward(ctypes.byref(scene.c()), ctypes.byref(proj.c()), _ptr(binned.vals),
                                       _ptr(binned.ranges), _ptr(binned.order), cameras(cams), V,
                                       ctypes.byref(opts.c()),
                                       _ptr(frame.t_final), _ptr(frame.last), _ptr(dl_dcolor.contiguous()),
                                       _ptr(active), _ptr(grad2d), ctypes.byref(_grads_c(grads)), _stream(stream)),
            "gs_render_backward")
    return grads, grad2d


def render_backward_pixels(proj: Projected, binned: Binned, cams, n: int, opts: RasterOpts, frame: Frame,
                           dl_dcolor: torch.Tensor, active=None, grad2d=None, stream=None,
                           deterministic: bool = False, det_ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Per-record 2D gradients (added into grad2d).  With `deterministic` the
    library's ordered reduction runs instead of float atomics (bitwise the same
    from run to run); `det_ws` may hold a reusable workspace for it."""
    V = len(cams)
    if grad2d is None:
        grad2d = torch.zeros((max(V * n, 1), L.GS_GRAD2D_FLOATS), device=proj.rec.device)
    if deterministic:
        ni = int(binned.stats.n_isect)
        need = max(L.lib().gs_render_backward_det_workspace_size(ni), 1)
        ws = det_ws if det_ws is not None and det_ws.numel() >= need else torch.empty(
            need, dtype=torch.uint8, device=proj.rec.device)
        L.check(L.lib().gs_render_backward_pixels_det(
            ctypes.byref(proj.c()), _ptr(binned.vals), _ptr(binned.ranges), _ptr(binned.order),
            _ptr(binned.offsets), cameras(cams), V, n, ni, ctypes.byref(opts.c()), _ptr(frame.t_final),
            _ptr(frame.last), _ptr(dl_dcolor.contiguous()), _ptr(active), _ptr(grad2d), _ptr(ws), ws.numel(),
            _stream(stream)), "gs_render_backward_pixels_det")
        return grad2d
    L.check(L.lib().gs_render_backward_pixels(ctypes.byref(proj.c()), _ptr(binned.vals), _ptr(binned.ranges),
                                              _ptr(binned.order), cameras(cams), V, n, ctypes.byref(opts.c()),
                                              _ptr(frame.t_final),
                                              _ptr(frame.last), _ptr(dl_dcolor.contiguous()), _ptr(active),
                                              _ptr(grad2d), _stream(stream)), "gs_render_backward_pixels")
    return grad2d


def fill_u32(t: torch.Tensor, value: int = 0, stream=None) -> None:
    """Fill a contiguous tensor of 4-byte elements with a 32-bit pattern
    (a kernel, not a memset: safe inside captured graphs)."""
    L.check(L.lib().gs_fill_u32(_ptr(t), value, t.numel() * t.element_size() // 4, _stream(stream)), "gs_fill_u32")


def l1_loss_grad(color: torch.Tensor, target: torch.Tensor, dl_dcolor: torch.Tensor, loss: Optional[torch.Tensor],
                 stream=None) -> None:
    L.check(L.lib().gs_l1_loss_grad(_ptr(color), _ptr(target), color.numel(), _ptr(dl_dcolor), _ptr(loss),
                                    _stream(stream)), "gs_l1_loss_grad")
