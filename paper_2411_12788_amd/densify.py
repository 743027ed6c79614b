"""Python binding of the culling and densification criteria (Sec. 5.1, Sec. 5.2,
Eq. (3)): argument marshalling only, every step runs in libmsplat.so."""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import torch

from . import _lib as L
from .raster import DeviceScene, Projected, _ptr, _stream, cameras, permute

KEEP_QUANTILE = 0.99   # Sec. 5.1 and Sec. 5.2
THETA_BLUR = 2e-4      # Eq. (3)
THRESHOLD_VALUE, THRESHOLD_MASS = L.GS_THRESHOLD_VALUE, L.GS_THRESHOLD_MASS


def _select_ws(problems: int, device) -> torch.Tensor:
    nbytes = L.lib().gs_select_workspace_size(problems)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def visibility(importance: torch.Tensor, keep: float = KEEP_QUANTILE, mode: int = THRESHOLD_MASS,
               ws: Optional[torch.Tensor] = None, stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """importance [V, n] float32 -> (visible [V, n] uint8, tau [V] float64)."""
    imp = importance if importance.dim() == 2 else importance.view(1, -1)
    assert imp.is_contiguous() and imp.dtype == torch.float32
    V, n = imp.shape
    visible = torch.empty((V, n), dtype=torch.uint8, device=imp.device)
    tau = torch.empty(V, dtype=torch.float64, device=imp.device)
    ws = _select_ws(V, imp.device) if ws is None else ws
    L.check(L.lib().gs_visibility(_ptr(imp), V, n, keep, mode, _ptr(visible), _ptr(tau), _ptr(ws), ws.numel(),
                                  _stream(stream)), "gs_visibility")
    return visible, tau


def critical(area: torch.Tensor, wmax: torch.Tensor, keep: float = KEEP_QUANTILE, mode: int = THRESHOLD_MASS,
             ws: Optional[torch.Tensor] = None, stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """area [n] int32/uint32, wmax [n] float32 -> (critical [n] uint8, tau [1] float64)."""
    assert area.is_contiguous() and area.element_size() == 4 and wmax.dtype == torch.float32
    n = wmax.numel()
    out = torch.empty(n, dtype=torch.uint8, device=wmax.device)
    tau = torch.empty(1, dtype=torch.float64, device=wmax.device)
    ws = _select_ws(1, wmax.device) if ws is None else ws
    L.check(L.lib().gs_critical(_ptr(area), _ptr(wmax), n, keep, mode, _ptr(out), _ptr(tau), _ptr(ws), ws.numel(),
                                _stream(stream)), "gs_critical")
    return out, tau


def blur_split(area: torch.Tensor, height: int, width: int, theta: float = THETA_BLUR, stream=None) -> torch.Tensor:
    n = area.numel()
    out = torch.empty(n, dtype=torch.uint8, device=area.device)
    L.check(L.lib().gs_blur_split(_ptr(area), n, theta, height, width, _ptr(out), _stream(stream)), "gs_blur_split")
    return out


def grad_stats(proj: Projected, grad2d: torch.Tensor, cams, n: int, norm_sum: torch.Tensor, count: torch.Tensor,
               stream=None) -> None:
    cc = cameras(cams)
    L.check(L.lib().gs_grad_stats(ctypes.byref(proj.c()), _ptr(grad2d), cc, len(cc), n, _ptr(norm_sum), _ptr(count),
                                  _stream(stream)), "gs_grad_stats")


def clone(scene: DeviceScene, select: torch.Tensor, capacity: Optional[int] = None,
          stream=None) -> Tuple[DeviceScene, torch.Tensor]:
    """Two-way clone of the selected rows (Sec. 5.1).  With capacity None the
    selected count is read back first (one synchronisation) to size the output."""
    n = scene.n
    dev = scene.opacity.device
    if capacity is None:
        capacity = n + int(select.sum().item())
    out = DeviceScene(torch.empty((3, capacity), device=dev), torch.empty((3, capacity), device=dev),
                      torch.empty((4, capacity), device=dev), torch.empty(capacity, device=dev),
                      torch.empty((16, 3, capacity), device=dev), scene.sh_degree)
    so = L.SceneOut(_ptr(out.means), _ptr(out.scales), _ptr(out.quats), _ptr(out.opacity), _ptr(out.sh), capacity)
    count = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(L.lib().gs_clone_workspace_size(n), dtype=torch.uint8, device=dev)
    L.check(L.lib().gs_clone(ctypes.byref(scene.c()), _ptr(select), ctypes.byref(so), _ptr(count), _ptr(ws),
                             ws.numel(), _stream(stream)), "gs_clone")
    return out, count


def reorder(scene: DeviceScene, *rows: torch.Tensor, stream=None):
    """(scene, [rows], perm): the scene and any per-Gaussian arrays (contiguous,
    last dimension n: optimizer moments, accumulated statistics, masks) moved
    into the library's spatial order, Gaussian i of the results being
    Gaussian perm[i] of the inputs.  For use after the set of Gaussians
    changes (clone, split, pruning), when appended rows have broken the
    order; a memory layout only, every result is the same up to perm."""
    out, perm = scene.in_spatial_order(stream)
    return out, [permute(t, perm, stream) for t in rows], perm


SPLIT_FACTOR = 1.6  # 3DGS: children take the parent's scales divided by 1.6


def densify_select(norm_sum: torch.Tensor, count: torch.Tensor, scales: torch.Tensor, grad_threshold: float,
                   scale_threshold: float, stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """(clone [n], split [n]) uint8 masks of the 3DGS density control (Sec. 3.2)."""
    n = norm_sum.numel()
    dev = norm_sum.device
    clone_m = torch.empty(n, dtype=torch.uint8, device=dev)
    split_m = torch.empty(n, dtype=torch.uint8, device=dev)
    L.check(L.lib().gs_densify_select(_ptr(norm_sum), _ptr(count), _ptr(scales), n, float(grad_threshold),
                                      float(scale_threshold), _ptr(clone_m), _ptr(split_m), _stream(stream)),
            "gs_densify_select")
    return clone_m, split_m


def split(scene: DeviceScene, select: torch.Tensor, normals: torch.Tensor, factor: float = SPLIT_FACTOR,
          capacity: Optional[int] = None, stream=None) -> Tuple[DeviceScene, torch.Tensor]:
    """Split of the selected rows into two children drawn from the parent
    (normals [2, 3, n] standard-normal draws); unselected rows first."""
    n = scene.n
    dev = scene.opacity.device
    if capacity is None:
        capacity = n + int(select.sum().item())
    out = DeviceScene(torch.empty((3, capacity), device=dev), torch.empty((3, capacity), device=dev),
                      torch.empty((4, capacity), device=dev), torch.empty(capacity, device=dev),
                      torch.empty((16, 3, capacity), device=dev), scene.sh_degree)
    so = L.SceneOut(_ptr(out.means), _ptr(out.scales), _ptr(out.quats), _ptr(out.opacity), _ptr(out.sh), capacity)
    count = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(L.lib().gs_split_workspace_size(n), dtype=torch.uint8, device=dev)
    L.check(L.lib().gs_split(ctypes.byref(scene.c()), _ptr(select), _ptr(normals), float(factor), ctypes.byref(so),
                             _ptr(count), _ptr(ws), ws.numel(), _stream(stream)), "gs_split")
    return out, count


def sample(importance: torch.Tensor, expo: torch.Tensor, k: int, area: Optional[torch.Tensor] = None,
           stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Intersection preserving + primitive sampling (Sec. 4.2): (selected [n] uint8, count [1] int64).
    expo holds Exp(1) draws, one per Gaussian."""
    n = importance.numel()
    dev = importance.device
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    count = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(L.lib().gs_sample_workspace_size(n), dtype=torch.uint8, device=dev)
    L.check(L.lib().gs_sample(_ptr(importance), _ptr(area), _ptr(expo), n, int(k), _ptr(out), _ptr(count), _ptr(ws),
                              ws.numel(), _stream(stream)), "gs_sample")
    return out, count


def depth_points(depth: torch.Tensor, imax: torch.Tensor, hit: Optional[torch.Tensor], target: torch.Tensor,
                 u: torch.Tensor, cams, rate: float, require_hit: bool = True, capacity: Optional[int] = None,
                 stream=None) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
    """Depth reinitialisation points (Sec. 4.1): (points [3, cap], colors [3, cap], count [1] int64)."""
    cc = cameras(cams)
    P = depth.numel()
    dev = depth.device
    cap = P if capacity is None else int(capacity)
    pts = torch.empty((3, cap), device=dev)
    col = torch.empty((3, cap), device=dev)
    count = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(L.lib().gs_depth_points_workspace_size(P), dtype=torch.uint8, device=dev)
    L.check(L.lib().gs_depth_points(_ptr(depth), _ptr(imax), _ptr(hit), _ptr(target), _ptr(u), cc, len(cc), rate,
                                    1 if require_hit else 0, _ptr(pts), _ptr(col), cap, _ptr(count), _ptr(ws),
                                    ws.numel(), _stream(stream)), "gs_depth_points")
    return pts, col, count
