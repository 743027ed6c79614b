"""Shared helpers for GPU parity tests: run the HIP path and the oracle on the
same seeded inputs and compare with the stated tolerances.

Every pixel is checked.  Where float32 and float64 may legitimately take a
different discrete decision of Eq. (1)-(2) (a pair's alpha next to the skip
threshold, a transmittance next to the stop threshold, two weights next to a
tie), the oracle evaluates every branch of those decisions and the GPU pixel
must equal one of them; everywhere else it must equal the definition.  The
branch each pixel took is then fed back to the oracle, so the per-Gaussian
accumulations and the gradients are compared with what the oracle computes
under the same decisions."""
from __future__ import annotations

import json
import os

import numpy as np
import torch

import oracle
from oracle import F

# Tolerances.
COLOR_ATOL = 1e-4        # colour, depth, transmittance: max abs
GRAD_REL_L2 = 1e-3       # per parameter group
# The projection backward alone (parameters from the per-record 2D gradient):
# its chain rule runs in float, ordered so that no intermediate cancels by
# more than the elongation of a Gaussian; emulated in float32 against float64
# on needles of elongation 12 its largest error is 4.2e-5 (scales).
A8_REL_L2 = 1e-4
# Relative widths inside which a decision is evaluated both ways.  Wider than
# the float32 error of the decision's operands:
# alpha is exp2 of a float32 exponent (error ~1e-6 relative); a transmittance
# after k factors carries ~k ulp plus up to 100x the alpha error of a factor
# with alpha near 0.99; weights carry the transmittance's error.
ALPHA_MARGIN = 2e-5
STOP_MARGIN = 2e-3
ARGMAX_MARGIN = 1e-4
AMB = (ALPHA_MARGIN, STOP_MARGIN, ARGMAX_MARGIN)
# the hit flag is a sign test of a double discriminant on both sides
HIT_MARGIN = 1e-9
# Per-Gaussian sums.  Tolerance derived from the arithmetic: the oracle gives
# per Gaussian the first-order float32 error bound of each weight w = alpha T
# (alpha from a float32 exponent; each factor 1 - alpha carries alpha's error
# magnified by alpha / (1 - alpha); one rounding per product), summed over the
# Gaussian's pairs for the importance, plus count * u * I for a float32 sum
# of `count` positive terms in any order; twice that bound, plus ACC_REL of
# the value, is allowed.
ACC_REL = 1e-6
ACC_BOUND_FACTOR = 2.0
U32 = 2.0 ** -24


def raster():
    from paper_2411_12788_amd import raster as R
    return R


def report(name, **vals):
    """Appends measured figures to the file named by GS_PARITY_REPORT (if set)."""
    path = os.environ.get("GS_PARITY_REPORT")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps({"case": name, **{k: (v.item() if hasattr(v, "item") else v)
                                                 for k, v in vals.items()}}) + "\n")


def gpu_opts(**kw):
    R = raster()
    return R.RasterOpts(**kw)


def run_gpu_forward(scene, cams, opts=None, cull=None, accumulate=True, per_view=False, want_keys=False):
    R = raster()
    opts = opts or R.RasterOpts()
    ds = R.DeviceScene.from_numpy(scene)
    cm = None if cull is None else torch.from_numpy(cull).cuda()
    proj = R.project(ds, cams, opts, cm)
    binned = R.bin(proj, cams, ds.n, want_keys=want_keys)
    acc = R.alloc_accum(ds.n, len(cams), per_view) if accumulate else None
    if accumulate and per_view:
        opts = R.RasterOpts(**{**opts.__dict__, "flags": opts.flags | 2})
    frame = R.render_forward(ds, proj, binned, cams, opts, accum=acc)
    torch.cuda.synchronize()
    return dict(scene=ds, proj=proj, binned=binned, frame=frame, acc=acc, opts=opts)


def gpu_pixels(frame, idx):
    """GPU per-pixel outputs at global pixel indices idx (numpy)."""
    it = torch.from_numpy(np.asarray(idx, dtype=np.int64)).cuda()
    out = dict(color=frame.color[:, it].T.double().cpu().numpy(),
               t_final=frame.t_final[it].double().cpu().numpy(),
               imax=frame.imax[it].long().cpu().numpy(),
               depth=frame.depth[it].double().cpu().numpy(),
               hit=frame.hit[it].cpu().numpy())
    out["n_contrib"] = frame.n_contrib[it].long().cpu().numpy() if frame.n_contrib is not None else None
    return out


def _agree(g, o, hit_margin):
    """Per pixel: GPU values g equal the oracle outcome o (arrays over pixels)."""
    ok = np.abs(g["color"] - o["color"]).max(axis=1) <= COLOR_ATOL
    ok &= np.abs(g["t_final"] - o["t_final"]) <= COLOR_ATOL
    if g["n_contrib"] is not None:
        ok &= g["n_contrib"] == o["n_contrib"]
    ok &= g["imax"] == o["imax"]
    ok &= np.abs(g["depth"] - o["depth"]) <= COLOR_ATOL
    ok &= (g["hit"] == o["hit"]) | (hit_margin < HIT_MARGIN)
    return ok


def match_pixels(gpu, orc, p, cam, proj, ordr, opts, pixels, what="", tiles=None):
    """Checks every pixel of a list: unambiguous pixels against the oracle's
    definition (orc = oracle.render at `pixels`), ambiguous ones against every
    branch.  Returns the flips of the branch each pixel matched (0 = the
    definition's decisions) and the count of ambiguous pixels.  ``tiles``
    (oracle binning of this view) restricts the oracle to each pixel's tile
    list, which the oracle's pins show changes nothing."""
    m = orc["margin"]
    amb = (m[:, 0] < AMB[0]) | (m[:, 1] < AMB[1]) | (m[:, 2] < AMB[2])
    flips = np.zeros(len(amb), dtype=np.uint32)
    plain = _agree(gpu, orc, m[:, 4])
    bad = np.nonzero(~plain & ~amb)[0]
    assert bad.size == 0, (what, "pixels differing from the definition", bad[:8].tolist(),
                           {k: (None if gpu[k] is None else gpu[k][bad[:3]].tolist()) for k in gpu},
                           {k: orc[k][bad[:3]].tolist() for k in ("color", "t_final", "n_contrib", "imax", "depth")})
    ai = np.nonzero(amb & ~plain)[0]
    if ai.size:
        pix = np.asarray(pixels, dtype=np.int32).reshape(-1, 2)[ai]
        br = oracle.branches(p, cam, proj, ordr, opts, pix, AMB, tiles=tiles)
        assert br["complete"].all(), (what, "too many branches")
        sub = {k: (None if v is None else v[ai]) for k, v in gpu.items()}
        found = np.zeros(ai.size, dtype=bool)
        for j in range(int(br["count"].max())):
            cand = {k: br[k][:, j] for k in ("color", "t_final", "n_contrib", "imax", "depth", "hit")}
            hm = br["margin"][:, j, 4]
            hitj = _agree(sub, cand, hm) & (j < br["count"]) & ~found
            flips[ai[hitj]] = br["flips"][hitj, j]
            found |= hitj
        miss = np.nonzero(~found)[0]
        assert miss.size == 0, (what, "pixels matching no branch", pix[miss[:8]].tolist(),
                                {k: (None if sub[k] is None else sub[k][miss[:3]].tolist()) for k in sub},
                                br["count"][miss[:8]].tolist())
    return flips, int(amb.sum())


def compare_forward(gpu_frame, orc, pix_slice, what, p, cam, opts=None):
    """Checks one view's GPU outputs against the oracle's full-image outputs
    (oracle.forward_view); returns the per-pixel flips and the ambiguous count."""
    opts = opts or oracle.Opts()
    W, H = int(cam.width), int(cam.height)
    ys, xs = np.divmod(np.arange(W * H), W)
    pixels = np.stack([xs, ys], 1).astype(np.int32)
    idx = np.arange(pix_slice.start, pix_slice.stop)
    gpu = gpu_pixels(gpu_frame, idx)
    flips, namb = match_pixels(gpu, orc, p, cam, orc["proj"], orc["order"], opts, pixels, what)
    report(what, pixels=W * H, ambiguous=namb, other_branch=int((flips != 0).sum()))
    return flips, namb


def check_accum(acc_g, p, cam, proj, ordr, opts, flips, n, what="", pixels=None, rows=None, tiles=None):
    """Per-Gaussian importance, max weight and area of the GPU against the
    oracle's, accumulated over the same pixels under the branch each pixel
    took.  Area exact; importance and max weight within the float32 error
    bound above, every Gaussian (or the given rows)."""
    o = oracle.render(p, cam, proj, ordr, opts, pixels=pixels, tiles=tiles, accumulate=True, amb=AMB, flips=flips)
    sel = np.arange(n) if rows is None else np.asarray(rows)
    acc_g = {k: (v.detach().cpu().numpy() if torch.is_tensor(v) else np.asarray(v)) for k, v in acc_g.items()}
    imp_g = acc_g["importance"][sel].astype(np.float64)
    wm_g = acc_g["wmax"][sel].astype(np.float64)
    ar_g = acc_g["area"][sel].astype(np.int64)
    imp_o, wm_o, ar_o = o["importance"][sel], o["wmax"][sel], o["area"][sel]
    tol = o["acc_tol"][sel]
    tol_i = ACC_REL * imp_o + ACC_BOUND_FACTOR * (tol[:, 0] + tol[:, 2] * U32 * imp_o) + 1e-30
    tol_w = ACC_REL * wm_o + ACC_BOUND_FACTOR * tol[:, 1] + 1e-30
    di, dw = np.abs(imp_g - imp_o), np.abs(wm_g - wm_o)
    ei = di / np.maximum(imp_o, 1e-30)
    ew = dw / np.maximum(wm_o, 1e-30)
    report(what + " accum", gaussians=len(sel), imp_rel_max=float(ei[imp_o > 0].max(initial=0)),
           wmax_rel_max=float(ew[wm_o > 0].max(initial=0)), imp_err_over_tol=float((di / tol_i).max(initial=0)),
           wmax_err_over_tol=float((dw / tol_w).max(initial=0)), area_mismatch=int((ar_g != ar_o).sum()))
    assert np.array_equal(ar_g, ar_o), (what, "area", np.nonzero(ar_g != ar_o)[0][:8].tolist())
    bi = np.nonzero(di > tol_i)[0]
    assert bi.size == 0, (what, "importance", bi[:8].tolist(), imp_g[bi[:4]].tolist(), imp_o[bi[:4]].tolist(),
                          tol_i[bi[:4]].tolist())
    bw = np.nonzero(dw > tol_w)[0]
    assert bw.size == 0, (what, "wmax", bw[:8].tolist(), wm_g[bw[:4]].tolist(), wm_o[bw[:4]].tolist(),
                          tol_w[bw[:4]].tolist())
    return o


def backward_views(p, cams, opts, dldc, active=None, flips=None):
    """Oracle parameter gradients of sum_v sum(dldc[v] * C_v) with each view's
    pixels taking the branch in flips[v] (full images, row-major)."""
    grads, g2ds = None, []
    for v, cam in enumerate(cams):
        proj = oracle.project(p, cam, opts)
        ordr = oracle.order(proj)
        g2d = oracle.render_backward(p, cam, proj, ordr, opts, dldc[v], amb=AMB,
                                     flips=None if flips is None else flips[v])
        g2ds.append(g2d)
        grads = oracle.project_backward(p, cam, opts, proj, g2d, grads)
    if active is not None:
        msk = np.asarray(active).astype(bool)
        for g in grads.values():
            g[..., ~msk] = 0.0
    return grads, g2ds


def view_slice(layout, v):
    lo = layout.pixel_base[v]
    return slice(lo, lo + (layout.pixel_base[v + 1] if v + 1 < len(layout.pixel_base) else layout.pixels_total) - lo)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def check_projection_backward(p, cams, opts, g2d, grads, n, active=None, what=""):
    """The GPU's parameter gradients against the oracle's projection backward
    applied to the GPU's own per-record 2D gradient g2d [V n, 9] (the
    projection backward alone, a8), group by group at A8_REL_L2."""
    g2d = np.asarray(g2d, dtype=np.float64)
    og = None
    for v, cam in enumerate(cams):
        proj = oracle.project(p, cam, opts)
        og = oracle.project_backward(p, cam, opts, proj, g2d[v * n:(v + 1) * n], og)
    if active is not None:
        msk = np.asarray(active).astype(bool)
        for g in og.values():
            g[..., ~msk] = 0.0
    errs = {}
    for k in ("means", "scales", "quats", "opacity", "sh"):
        got = np.asarray(grads[k], dtype=np.float64)[..., :n]
        errs[k] = rel_l2(got, og[k])
    report(f"projection backward alone {what}", **errs)
    for k, e in errs.items():
        assert e <= A8_REL_L2, (what, k, e)
    return errs


def check_bin_extras(b, rects, zb, n_views, tiles_total, ranges, what=""):
    """The count's side outputs and the tile order against their definitions
    over the oracle's tile rectangles and depth bits: offsets = exclusive scan
    of the tiles each record touches; n_visible = records touching a tile;
    zbits_min / max over those; depth_bits = bit length of their spread;
    key_bits = depth_bits + bit length of (tiles_total - 1); the tile order =
    lists by descending bit length of their length, ascending tile id inside
    one bit length (`ranges` are the oracle's [tiles_total, 2])."""
    r = np.asarray(rects, dtype=np.int64)
    cnt = np.where((r[:, 0] <= r[:, 1]) & (r[:, 2] <= r[:, 3]), (r[:, 1] - r[:, 0] + 1) * (r[:, 3] - r[:, 2] + 1), 0)
    assert cnt.sum() < 2 ** 32
    want_off = (np.cumsum(cnt) - cnt).astype(np.uint32)
    got_off = b.offsets.cpu().numpy().view(np.uint32)[: len(cnt)]
    bad = np.flatnonzero(got_off != want_off)
    assert bad.size == 0, (what, "offsets", bad[:8].tolist())
    st = b.stats
    vis = cnt > 0
    assert st.n_isect == int(cnt.sum()), what
    assert st.n_visible == int(vis.sum()), (what, st.n_visible, int(vis.sum()))
    zv = np.asarray(zb, dtype=np.uint32)[vis]
    zmin, zmax = (int(zv.min()), int(zv.max())) if zv.size else (0, 0)
    assert (st.zbits_min, st.zbits_max) == (zmin, zmax), (what, st.zbits_min, st.zbits_max, zmin, zmax)
    assert st.depth_bits == (zmax - zmin).bit_length(), what
    assert st.key_bits == st.depth_bits + (tiles_total - 1).bit_length(), what
    if b.order is not None:
        L = (ranges[:, 1].astype(np.int64) - ranges[:, 0].astype(np.int64))
        bits = np.array([int(x).bit_length() for x in L])
        want = np.lexsort((np.arange(len(L)), -bits))
        got = b.order.cpu().numpy().view(np.uint32).astype(np.int64)
        assert np.array_equal(got, want), (what, "tile order", int((got != want).sum()))
