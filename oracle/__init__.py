"""FP64 CPU oracle for differentiable tile-based Gaussian rasterization.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP path (``paper_2411_12788_amd``); the only module both sides
read is ``gs_inputs`` (seeded input draws, no rasterizer arithmetic).

The arithmetic lives in ``oracle.c`` (plain C, double precision, one pixel and
one Gaussian at a time); this file only marshals numpy arrays.  Each function
cites the passage of the paper it follows; the pins that tie it to something
other than itself live in ``tests/test_oracle_*.py``:

  project           Sec. 3.1 (EWA projection, SH colour)   pinned: closed forms,
                    Monte-Carlo covariance, SH vs scipy + quadrature, FD
  order             Sec. 3.1 (approximate depth order)     pinned: numpy lexsort
  render            Eq. (1), Eq. (2), Sec. 4.1 mid-point depth, Sec. 3.2
                    importance, Eq. (3) area, Sec. 5.1 w_imax
                                                           pinned: closed forms,
                    invariants, tiled == untiled, golden-section depth, brute force
  render_backward   derivative of Eq. (1)                  pinned: central FD
  project_backward  derivative of Sec. 3.1 projection      pinned: central FD
  bin               tile | depth keys, stable sort, ranges pinned: numpy lexsort
  quantile, visibility, critical, blur_split, clone
                    Sec. 5.1, Sec. 5.2, Eq. (3)             pinned: numpy quantile,
                    two-clone opacity identity, small-opacity limit, paper constants
  depth_points      Sec. 4.1 (reprojection of the depth map)  pinned: projection round trip
  sample            Sec. 4.2 (intersection preserving, primitive sampling)
                                                            pinned: exact inclusion probabilities
                                                            of sequential weighted draws
  densify_select, split
                    Sec. 3.2 / Sec. 4.1 (3DGS density control; blur split
                    children)                               pinned: closed-form rotations,
                    covariance of the children vs scipy's rotation, boundary cases
  tile_alpha_max    Eq. (1) alpha over a tile's pixel centres (tile culling checks)
                                                            pinned: isotropic closed form,
                    centre inside the tile
  spatial_order     not a step of the method: the GPU library's memory layout
                    (Morton order of the means), checked so that its permutation
                    is exact                                pinned: octree descent in
                    double, Z-order of grid points, numpy stable argsort, special cases
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import build as _build

HERE = os.path.dirname(os.path.abspath(__file__))
STRIDE = 32
# projected record fields (mirrors the enum in oracle.c)
F = dict(VALID=0, U=1, V=2, Z=3, CA=4, CB=5, CC=6, S00=7, S01=8, S11=9, R=10, G=11, B=12,
         RAW_R=13, RAW_G=14, RAW_B=15, OPAC=16, RX=17, RY=18, XLO=19, XHI=20, YLO=21, YHI=22,
         TILES=23, TXTZ=24, TYTZ=25, ZF=26)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = ctypes.CDLL(_build.LIB)
        _lib.orc_order.restype = ctypes.c_int64
        _lib.orc_bin.restype = ctypes.c_int64
        _lib.orc_quantile.restype = ctypes.c_double
        _lib.orc_visibility.restype = ctypes.c_double
        _lib.orc_threshold.restype = ctypes.c_double
        _lib.orc_mass_threshold.restype = ctypes.c_double
        _lib.orc_critical.restype = ctypes.c_double
        _lib.orc_clone.restype = ctypes.c_int64
        _lib.orc_depth_points.restype = ctypes.c_int64
        _lib.orc_sample.restype = ctypes.c_int64
        _lib.orc_split.restype = ctypes.c_int64
    return _lib


class OCam(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class OOpts(ctypes.Structure):
    _fields_ = [("znear", ctypes.c_double), ("lowpass", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("alpha_min", ctypes.c_double), ("t_min", ctypes.c_double), ("jac_clamp", ctypes.c_double),
                ("bg", ctypes.c_double * 3), ("depth_mode", ctypes.c_int32), ("tile", ctypes.c_int32)]


def _f32(x: float) -> float:
    return float(np.float32(x))


@dataclasses.dataclass
class Opts:
    """Rasterizer constants.  The paper states none of them; these are the
    float32 values of the 3DGS-lineage constants (alpha clamp 0.99, skip below
    1/255, stop below transmittance 1e-4, low-pass 0.3, Jacobian clamp 1.3,
    near plane 0.2, 16x16 tiles)."""
    znear: float = _f32(0.2)
    lowpass: float = _f32(0.3)
    alpha_max: float = _f32(0.99)
    alpha_min: float = _f32(1.0 / 255.0)
    t_min: float = _f32(1e-4)
    jac_clamp: float = _f32(1.3)
    bg: Sequence[float] = (0.0, 0.0, 0.0)
    depth_mode: int = 0  # 0 mid-point, 1 centre, 2 blended
    tile: int = 16

    def c(self) -> OOpts:
        o = OOpts()
        o.znear, o.lowpass, o.alpha_max = self.znear, self.lowpass, self.alpha_max
        o.alpha_min, o.t_min, o.jac_clamp = self.alpha_min, self.t_min, self.jac_clamp
        for k in range(3):
            o.bg[k] = float(self.bg[k])
        o.depth_mode, o.tile = int(self.depth_mode), int(self.tile)
        return o


def ocam(cam) -> OCam:
    c = OCam()
    R = np.asarray(cam.R, dtype=np.float64).reshape(9)
    t = np.asarray(cam.t, dtype=np.float64).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray):
    # the C side indexes plain row-major arrays: a strided view (a column slice
    # of a [k][n] plane array, say) would be read with the wrong layout
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("oracle: arrays passed to the C oracle must be C-contiguous")
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclasses.dataclass
class Params:
    """Scene parameters in float64 (widened float32 inputs, or perturbed copies)."""
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray
    sh_degree: int

    def __post_init__(self):
        # contiguous float64 planes (slices of another Params are copied)
        for k in ("means", "scales", "quats", "opacity", "sh"):
            setattr(self, k, _d(getattr(self, k)))

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])

    @staticmethod
    def of(scene) -> "Params":
        return Params(_d(scene.means), _d(scene.scales), _d(scene.quats), _d(scene.opacity),
                      _d(scene.sh), int(scene.sh_degree))

    def copy(self) -> "Params":
        return Params(self.means.copy(), self.scales.copy(), self.quats.copy(), self.opacity.copy(),
                      self.sh.copy(), self.sh_degree)


def project(params: Params, cam, opts: Opts, cull_mask: Optional[np.ndarray] = None) -> np.ndarray:
    """Per-Gaussian projection of one view [Sec. 3.1]; returns proj[n, STRIDE]."""
    n = params.n
    proj = np.zeros((max(n, 1), STRIDE), dtype=np.float64)
    cm = None if cull_mask is None else np.ascontiguousarray(cull_mask, dtype=np.uint8)
    c, o = ocam(cam), opts.c()
    lib().orc_project(ctypes.c_int64(n), _p(params.means), _p(params.scales), _p(params.quats),
                      _p(params.opacity), _p(params.sh), ctypes.c_int(params.sh_degree), ctypes.byref(c),
                      None if cm is None else _p(cm), ctypes.byref(o), _p(proj))
    return proj[:n]


def order(proj: np.ndarray) -> np.ndarray:
    """Valid records by (float32 bits of camera depth, index) [Sec. 3.1]."""
    n = proj.shape[0]
    out = np.zeros(max(n, 1), dtype=np.int64)
    m = lib().orc_order(ctypes.c_int64(n), _p(np.ascontiguousarray(proj)), _p(out))
    return out[:m]


def _amb(amb) -> Optional[np.ndarray]:
    return None if amb is None else _d(amb).reshape(3)


def render(params: Params, cam, proj: np.ndarray, ordr: np.ndarray, opts: Opts,
           pixels: Optional[np.ndarray] = None, tiles=None, accumulate: bool = True,
           amb=None, flips: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """Eq. (1) compositing with Eq. (2) argmax depth and the per-Gaussian sums.

    ``pixels``: optional int32 [m, 2] (x, y) list; default every pixel, row-major.
    ``tiles``: optional (vals, ranges) from :func:`bin` to restrict each pixel to
    its tile's list.  ``margin`` columns: alpha vs skip threshold, transmittance
    vs stop threshold, top-two weight gap, opacity*G vs clamp, and the relative
    ray/ellipsoid discriminant of the hit flag (all relative).
    ``amb`` (alpha, stop, argmax widths) and ``flips`` (uint32 per pixel) invert
    the decisions that lie within those widths of their thresholds (bit k of
    ``flips`` for the k-th such decision met); ``namb`` returns how many were met.
    With ``accumulate``, ``acc_tol`` [n, 3] holds per Gaussian the first-order
    float32 error bounds of the importance terms and of the max weight, and the
    number of included pairs (test tolerances; see oracle.c).
    """
    n = params.n
    W, H = int(cam.width), int(cam.height)
    pix = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int32)
    npx = W * H if pix is None else pix.shape[0]
    out = dict(color=np.zeros((npx, 3)), depth=np.zeros(npx), imax=np.zeros(npx, dtype=np.int64),
               t_final=np.zeros(npx), n_contrib=np.zeros(npx, dtype=np.int32),
               hit=np.zeros(npx, dtype=np.uint8), margin=np.zeros((npx, 5)), namb=np.zeros(npx, dtype=np.int32))
    if accumulate:
        out.update(importance=np.zeros(max(n, 1)), wmax=np.zeros(max(n, 1)),
                   area=np.zeros(max(n, 1), dtype=np.int64), acc_tol=np.zeros((max(n, 1), 3)))
    tv = tr = None
    if tiles is not None:
        tv = np.ascontiguousarray(tiles[0], dtype=np.uint32)
        tr = np.ascontiguousarray(tiles[1], dtype=np.uint32)
    a = _amb(amb)
    fl = None if flips is None else np.ascontiguousarray(flips, dtype=np.uint32).reshape(npx)
    c, o = ocam(cam), opts.c()
    ordr = np.ascontiguousarray(ordr, dtype=np.int64)
    rc = lib().orc_render_ex(
        ctypes.c_int64(n), _p(np.ascontiguousarray(proj)), _p(ordr), ctypes.c_int64(len(ordr)),
        _p(params.means), _p(params.scales), _p(params.quats), ctypes.byref(c), ctypes.byref(o),
        ctypes.c_int64(npx), None if pix is None else _p(pix), None if tv is None else _p(tv),
        None if tr is None else _p(tr), None if a is None else _p(a), None if fl is None else _p(fl),
        _p(out["namb"]), _p(out["color"]), _p(out["depth"]), _p(out["imax"]),
        _p(out["t_final"]), _p(out["n_contrib"]), _p(out["hit"]), _p(out["margin"]),
        _p(out["importance"]) if accumulate else None, _p(out["wmax"]) if accumulate else None,
        _p(out["area"]) if accumulate else None, _p(out["acc_tol"]) if accumulate else None)
    assert rc == 0
    if accumulate:
        for k in ("importance", "wmax", "area", "acc_tol"):
            out[k] = out[k][:n]
    return out


def branches(params: Params, cam, proj: np.ndarray, ordr: np.ndarray, opts: Opts, pixels: np.ndarray,
             amb, max_branches: int = 64, tiles=None) -> Dict[str, np.ndarray]:
    """Every outcome of Eq. (1)-(2) at the given pixels when each decision that
    lies within ``amb`` of its threshold may go either way (test support for a
    float32 renderer).  Flip masks are enumerated in increasing order; a mask is
    a distinct branch when it sets no bit beyond the ambiguous decisions its own
    path meets, and the masks below 2^(most decisions met on any branch) cover
    every branch.  Returns per pixel ``count`` and, for branch j < count, the
    arrays ``flips``, ``color``, ``t_final``, ``n_contrib``, ``imax``, ``depth``,
    ``hit`` and ``margin`` with a leading [m, max_branches] shape; ``complete``
    is False for a pixel with more than max_branches branches.  ``tiles`` as in
    :func:`render`."""
    pix = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
    m, B = pix.shape[0], int(max_branches)
    res = dict(count=np.zeros(m, dtype=np.int64), complete=np.ones(m, dtype=bool),
               flips=np.zeros((m, B), dtype=np.uint32), color=np.zeros((m, B, 3)), t_final=np.zeros((m, B)),
               n_contrib=np.zeros((m, B), dtype=np.int32), imax=np.zeros((m, B), dtype=np.int64),
               depth=np.zeros((m, B)), hit=np.zeros((m, B), dtype=np.uint8), margin=np.zeros((m, B, 5)))
    need = np.ones(m, dtype=np.int64)  # 2^(most ambiguous decisions met so far), per pixel
    mask = 0
    while True:
        todo = np.nonzero(mask < need)[0]
        if todo.size == 0:
            break
        r = render(params, cam, proj, ordr, opts, pixels=pix[todo], tiles=tiles, accumulate=False, amb=amb,
                   flips=np.full(todo.size, mask, dtype=np.uint32))
        d = r["namb"].astype(np.int64)
        valid = (mask >> np.minimum(d, 62)) == 0
        need[todo] = np.maximum(need[todo], np.left_shift(1, np.minimum(d, 62)))
        for j in np.nonzero(valid)[0]:
            p = todo[j]
            c = res["count"][p]
            if c >= B:
                res["complete"][p] = False
                continue
            res["flips"][p, c] = mask
            for k in ("color", "t_final", "n_contrib", "imax", "depth", "hit", "margin"):
                res[k][p, c] = r[k][j]
            res["count"][p] = c + 1
        mask += 1
        if mask >= (1 << 20):
            res["complete"][todo] = False
            break
    return res


def render_backward(params: Params, cam, proj: np.ndarray, ordr: np.ndarray, opts: Opts,
                    dldc: np.ndarray, pixels: Optional[np.ndarray] = None, amb=None,
                    flips: Optional[np.ndarray] = None, tiles=None) -> np.ndarray:
    """Gradient of sum(dldc * C) w.r.t. each record's (u, v, a, b, c, opacity, r, g, b).

    ``dldc`` is [m, 3] for the pixel list (or [H*W, 3] row-major).  ``amb`` and
    ``flips`` select a decision branch per pixel, and ``tiles`` restricts each
    pixel to its tile's list, as in :func:`render`."""
    n = params.n
    pix = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int32)
    npx = int(cam.width) * int(cam.height) if pix is None else pix.shape[0]
    g = _d(dldc).reshape(npx, 3)
    g2d = np.zeros((max(n, 1), 9))
    a = _amb(amb)
    fl = None if flips is None else np.ascontiguousarray(flips, dtype=np.uint32).reshape(npx)
    tv = tr = None
    if tiles is not None:
        tv = np.ascontiguousarray(tiles[0], dtype=np.uint32)
        tr = np.ascontiguousarray(tiles[1], dtype=np.uint32)
    c, o = ocam(cam), opts.c()
    ordr = np.ascontiguousarray(ordr, dtype=np.int64)
    rc = lib().orc_render_backward_ex(ctypes.c_int64(n), _p(np.ascontiguousarray(proj)), _p(ordr),
                                      ctypes.c_int64(len(ordr)), ctypes.byref(c), ctypes.byref(o),
                                      ctypes.c_int64(npx), None if pix is None else _p(pix),
                                      None if tv is None else _p(tv), None if tr is None else _p(tr),
                                      None if a is None else _p(a), None if fl is None else _p(fl), _p(g), _p(g2d))
    assert rc == 0
    return g2d[:n]


def project_backward(params: Params, cam, opts: Opts, proj: np.ndarray, g2d: np.ndarray,
                     grads: Optional[Dict[str, np.ndarray]] = None) -> Dict[str, np.ndarray]:
    """Chain rule of :func:`project` (adds into ``grads``; sums over views when reused)."""
    n = params.n
    if grads is None:
        grads = dict(means=np.zeros((3, n)), scales=np.zeros((3, n)), quats=np.zeros((4, n)),
                     opacity=np.zeros(n), sh=np.zeros((16, 3, n)))
    c, o = ocam(cam), opts.c()
    rc = lib().orc_project_backward(
        ctypes.c_int64(n), _p(params.means), _p(params.scales), _p(params.quats), _p(params.opacity),
        _p(params.sh), ctypes.c_int(params.sh_degree), ctypes.byref(c), ctypes.byref(o),
        _p(np.ascontiguousarray(proj)), _p(_d(g2d)), _p(grads["means"]), _p(grads["scales"]),
        _p(grads["quats"]), _p(grads["opacity"]), _p(grads["sh"]))
    assert rc == 0
    return grads


def sh_basis(d: np.ndarray, degree: int = 3) -> np.ndarray:
    Y = np.zeros(16)
    lib().orc_sh_basis(_p(_d(d)), ctypes.c_int(degree), _p(Y))
    return Y


def sh_basis_grad(d: np.ndarray, degree: int = 3) -> np.ndarray:
    dY = np.zeros((16, 3))
    lib().orc_sh_basis_grad(_p(_d(d)), ctypes.c_int(degree), _p(dY))
    return dY


# ---------------------------------------------------------------------------------
# binning
# ---------------------------------------------------------------------------------
def view_layout(cams: Sequence, tile: int = 16):
    """Per-view tile grid: tiles_x[v], tiles_y[v], tile_base[v] (prefix sum), total."""
    tx = np.array([(int(c.width) + tile - 1) // tile for c in cams], dtype=np.int64)
    ty = np.array([(int(c.height) + tile - 1) // tile for c in cams], dtype=np.int64)
    base = np.concatenate([[0], np.cumsum(tx * ty)[:-1]]).astype(np.int64)
    return tx, ty, base, int((tx * ty).sum())


def tile_rects(proj: np.ndarray, tile: int = 16) -> np.ndarray:
    """(tx_lo, tx_hi, ty_lo, ty_hi) per record from the pixel box; empty -> (1, 0, 1, 0)."""
    n = proj.shape[0]
    out = np.tile(np.array([1, 0, 1, 0], dtype=np.int32), (n, 1))
    ok = (proj[:, F["VALID"]] != 0) & (proj[:, F["XLO"]] <= proj[:, F["XHI"]]) & \
         (proj[:, F["YLO"]] <= proj[:, F["YHI"]])
    box = proj[ok][:, [F["XLO"], F["XHI"], F["YLO"], F["YHI"]]].astype(np.int64)
    out[ok] = (box // tile).astype(np.int32)
    return out


def zbits(proj: np.ndarray) -> np.ndarray:
    return proj[:, F["Z"]].astype(np.float32).view(np.uint32)


def bin(rects: np.ndarray, zb: np.ndarray, n_views: int, n_per_view: int, tile_base, tiles_x,
        tiles_total: int):
    """Tile | depth keys, stable sort, per-tile ranges (integer work only)."""
    rects = np.ascontiguousarray(rects, dtype=np.int32)
    zb = np.ascontiguousarray(zb, dtype=np.uint32)
    tb = np.ascontiguousarray(tile_base, dtype=np.int64)
    tx = np.ascontiguousarray(tiles_x, dtype=np.int64)
    L = lib()
    total = L.orc_bin(ctypes.c_int64(n_views), ctypes.c_int64(n_per_view), _p(rects), _p(zb), _p(tb), _p(tx),
                      ctypes.c_int64(tiles_total), None, None, None)
    keys = np.zeros(max(total, 1), dtype=np.uint64)
    vals = np.zeros(max(total, 1), dtype=np.uint32)
    ranges = np.zeros(2 * max(tiles_total, 1), dtype=np.uint32)
    L.orc_bin(ctypes.c_int64(n_views), ctypes.c_int64(n_per_view), _p(rects), _p(zb), _p(tb), _p(tx),
              ctypes.c_int64(tiles_total), _p(keys), _p(vals), _p(ranges))
    return keys[:total], vals[:total], ranges[: 2 * tiles_total].reshape(tiles_total, 2)


# ---------------------------------------------------------------------------------
# whole-path conveniences
# ---------------------------------------------------------------------------------
def forward_view(params: Params, cam, opts: Opts, cull_mask=None, pixels=None, accumulate=True):
    proj = project(params, cam, opts, cull_mask)
    ordr = order(proj)
    out = render(params, cam, proj, ordr, opts, pixels=pixels, accumulate=accumulate)
    out["proj"], out["order"] = proj, ordr
    return out


def backward_views(params: Params, cams: Sequence, opts: Opts, dldc: List[np.ndarray],
                   active: Optional[np.ndarray] = None, cull_mask=None):
    """Parameter gradients of sum_v sum(dldc[v] * C_v); with ``active`` the rows
    of inactive Gaussians are zero (region-prioritized backward)."""
    grads = None
    g2ds = []
    for v, cam in enumerate(cams):
        proj = project(params, cam, opts, cull_mask)
        ordr = order(proj)
        g2d = render_backward(params, cam, proj, ordr, opts, dldc[v])
        g2ds.append(g2d)
        grads = project_backward(params, cam, opts, proj, g2d, grads)
    if active is not None:
        m = np.asarray(active).astype(bool)
        for k, g in grads.items():
            g[..., ~m] = 0.0
    return grads, g2ds


# ---------------------------------------------------------------------------------
# criteria consuming the accumulations (Sec. 5.1, Sec. 5.2, Eq. (3))
# ---------------------------------------------------------------------------------
KEEP_QUANTILE = 0.99   # Sec. 5.1 and Sec. 5.2
THETA_BLUR = 2e-4      # Eq. (3)


def quantile(values, q: float, mask=None) -> float:
    v = _d(values)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    return lib().orc_quantile(ctypes.c_int64(v.shape[0]), _p(v), None if m is None else _p(m), ctypes.c_double(q))


THRESHOLD_VALUE, THRESHOLD_MASS = 0, 1


def threshold(values, keep: float = KEEP_QUANTILE, mode: int = THRESHOLD_MASS, mask=None):
    """(tau, margin): the keep-quantile threshold of the selected values."""
    v = _d(values)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    margin = ctypes.c_double(0.0)
    tau = lib().orc_threshold(ctypes.c_int64(v.shape[0]), _p(v), None if m is None else _p(m), ctypes.c_double(keep),
                              ctypes.c_int(mode), ctypes.byref(margin))
    return tau, margin.value


def visibility(importance, keep: float = KEEP_QUANTILE, mode: int = THRESHOLD_MASS):
    """(visible[n] uint8, tau, margin) for one view's importances."""
    v = _d(importance)
    out = np.zeros(max(v.shape[0], 1), dtype=np.uint8)
    margin = ctypes.c_double(0.0)
    tau = lib().orc_visibility(ctypes.c_int64(v.shape[0]), _p(v), ctypes.c_double(keep), ctypes.c_int(mode), _p(out),
                               ctypes.byref(margin))
    return out[: v.shape[0]], tau, margin.value


def critical(area, wmax, keep: float = KEEP_QUANTILE, mode: int = THRESHOLD_MASS):
    """(critical[n] uint8, tau, margin)."""
    a = np.ascontiguousarray(area, dtype=np.int64)
    w = _d(wmax)
    out = np.zeros(max(a.shape[0], 1), dtype=np.uint8)
    margin = ctypes.c_double(0.0)
    tau = lib().orc_critical(ctypes.c_int64(a.shape[0]), _p(a), _p(w), ctypes.c_double(keep), ctypes.c_int(mode),
                             _p(out), ctypes.byref(margin))
    return out[: a.shape[0]], tau, margin.value


def blur_split(area, height: int, width: int, theta: float = THETA_BLUR):
    a = np.ascontiguousarray(area, dtype=np.int64)
    out = np.zeros(max(a.shape[0], 1), dtype=np.uint8)
    lib().orc_blur_split(ctypes.c_int64(a.shape[0]), _p(a), ctypes.c_double(theta), ctypes.c_int64(height),
                         ctypes.c_int64(width), _p(out))
    return out[: a.shape[0]]


def clone(params: Params, select) -> Params:
    sel = np.ascontiguousarray(select, dtype=np.uint8)
    n = params.n
    m = n + int(sel.sum())
    out = Params(np.zeros((3, m)), np.zeros((3, m)), np.zeros((4, m)), np.zeros(m), np.zeros((16, 3, m)),
                 params.sh_degree)
    lib().orc_clone(ctypes.c_int64(n), _p(params.means), _p(params.scales), _p(params.quats), _p(params.opacity),
                    _p(params.sh), _p(sel), _p(out.means), _p(out.scales), _p(out.quats), _p(out.opacity),
                    _p(out.sh))
    return out


def grad_stats(tiles, grad2d, widths, heights):
    """(norm_sum[n], count[n]) from tiles[V, n], grad2d[V * n, 9] (Sec. 3.2)."""
    t = np.ascontiguousarray(tiles, dtype=np.int32)
    V, n = t.shape
    g = _d(grad2d).reshape(V * n, 9)
    w = np.ascontiguousarray(widths, dtype=np.int32)
    h = np.ascontiguousarray(heights, dtype=np.int32)
    ns = np.zeros(max(n, 1))
    cnt = np.zeros(max(n, 1), dtype=np.int64)
    lib().orc_grad_stats(ctypes.c_int32(V), ctypes.c_int64(n), _p(t), _p(g), _p(w), _p(h), _p(ns), _p(cnt))
    return ns[:n], cnt[:n]


def tile_alpha_max(proj_row: np.ndarray, tx: int, ty: int, tile: int = 16) -> float:
    """Largest alpha = opacity * exp(-d^T conic d / 2) (Eq. (1)'s per-Gaussian
    alpha before the clamp) of one projected record over the pixel centres of
    tile (tx, ty) that lie in the record's pixel box; 0 if there are none.
    Brute force over the at most tile x tile pixels."""
    P = np.asarray(proj_row, dtype=np.float64)
    x0, x1 = max(tx * tile, int(P[F["XLO"]])), min(tx * tile + tile - 1, int(P[F["XHI"]]))
    y0, y1 = max(ty * tile, int(P[F["YLO"]])), min(ty * tile + tile - 1, int(P[F["YHI"]]))
    if x0 > x1 or y0 > y1:
        return 0.0
    xs = np.arange(x0, x1 + 1) + 0.5 - P[F["U"]]
    ys = np.arange(y0, y1 + 1) + 0.5 - P[F["V"]]
    dx, dy = np.meshgrid(xs, ys)
    q = P[F["CA"]] * dx * dx + 2.0 * P[F["CB"]] * dx * dy + P[F["CC"]] * dy * dy
    return float(P[F["OPAC"]] * np.exp(-0.5 * q.min()))


SPLIT_FACTOR = 1.6  # 3DGS: children take the parent's scales divided by 1.6


def densify_select(norm_sum, count, scales, grad_threshold: float, scale_threshold: float):
    """(clone[n], split[n]) of the 3DGS density control (Sec. 3.2): mean
    gradient norm >= grad_threshold, then largest scale <= / > scale_threshold."""
    ns = _d(norm_sum).ravel()
    n = ns.size
    cnt = np.ascontiguousarray(count, dtype=np.int64).ravel()
    sc = _d(scales).reshape(3, n)
    cl = np.zeros(max(n, 1), dtype=np.uint8)
    sp = np.zeros(max(n, 1), dtype=np.uint8)
    lib().orc_densify_select(ctypes.c_int64(n), _p(ns), _p(cnt), _p(sc), ctypes.c_double(grad_threshold),
                             ctypes.c_double(scale_threshold), _p(cl), _p(sp))
    return cl[:n].astype(bool), sp[:n].astype(bool)


def split(params: Params, select, normals, factor: float = SPLIT_FACTOR) -> Params:
    """3DGS split into two children drawn from the parent (normals[2, 3, n]
    standard-normal draws); unselected rows first, then the children."""
    sel = np.ascontiguousarray(select, dtype=np.uint8)
    n = params.n
    z = _d(normals).reshape(2, 3, n)
    m = n + int(sel.sum())
    out = Params(np.zeros((3, m)), np.zeros((3, m)), np.zeros((4, m)), np.zeros(m), np.zeros((16, 3, m)),
                 params.sh_degree)
    lib().orc_split(ctypes.c_int64(n), _p(params.means), _p(params.scales), _p(params.quats), _p(params.opacity),
                    _p(params.sh), _p(sel), _p(z), ctypes.c_double(factor), _p(out.means), _p(out.scales),
                    _p(out.quats), _p(out.opacity), _p(out.sh))
    return out


def depth_points(cam, depth, imax, hit, target, u, rate: float, require_hit: bool = True):
    """(points[m, 3], colors[m, 3]) lifted from one view's depth map (Sec. 4.1)."""
    P = int(cam.width) * int(cam.height)
    d = _d(depth).reshape(P)
    im = np.ascontiguousarray(imax, dtype=np.int32).reshape(P)
    h = np.ascontiguousarray(hit, dtype=np.int32).reshape(P)
    tg = _d(target).reshape(3, P)
    uu = _d(u).reshape(P)
    pts = np.zeros((max(P, 1), 3))
    col = np.zeros((max(P, 1), 3))
    c = ocam(cam)
    m = lib().orc_depth_points(ctypes.byref(c), _p(d), _p(im), _p(h), _p(tg), _p(uu), ctypes.c_double(rate),
                               ctypes.c_int(1 if require_hit else 0), _p(pts), _p(col))
    return pts[:m], col[:m]


def sample(importance, expo, k: int, area=None):
    """selected[n] uint8: k Gaussians drawn without replacement with probability
    proportional to importance, within area > 0 when area is given (Sec. 4.2)."""
    imp = np.ascontiguousarray(importance, dtype=np.float32)
    e = np.ascontiguousarray(expo, dtype=np.float32)
    a = None if area is None else np.ascontiguousarray(area, dtype=np.uint32)
    n = imp.shape[0]
    out = np.zeros(max(n, 1), dtype=np.uint8)
    lib().orc_sample(ctypes.c_int64(n), _p(imp), None if a is None else _p(a), _p(e), ctypes.c_int64(k), _p(out))
    return out[:n]


def spatial_order(means):
    """(codes[n] uint32, perm[n] int64): 30-bit Morton codes of the means
    [3, n] on a 1024^3 grid over the bounding box of the finite means, in
    float32, and the Gaussians in ascending code (ties: ascending index).  Not
    a step of the method: the memory order the GPU library keeps Gaussians in."""
    m = np.ascontiguousarray(means, dtype=np.float32)
    assert m.ndim == 2 and m.shape[0] == 3
    n = m.shape[1]
    codes = np.zeros(max(n, 1), dtype=np.uint32)
    perm = np.zeros(max(n, 1), dtype=np.int64)
    lib().orc_spatial_order(ctypes.c_int64(n), _p(m), _p(codes), _p(perm))
    return codes[:n], perm[:n]
