"""Parity at full workload sizes, in the launch configuration the benchmark
times: 3M Gaussians at 1920x1080 and 500k at 1245x825, and 1M Gaussians over
16 mixed-resolution views in one launch per stage.  The binning is compared
bit-exact in full; the oracle computes sampled outputs one by one: pixels over
every Gaussian, and for 50 sampled Gaussians per scene (small and large pixel
boxes, and Gaussians of the longest tile lists, which take the renderer's
split path) every pixel of the box over its tile's list, giving the
Gaussian's sums and 2D gradient.  Every sampled pixel is checked (ambiguous
decisions against each branch), and the oracle's sums and gradients follow
the branch each pixel took."""
import numpy as np
import pytest
import torch

import gs_inputs
import oracle
from oracle import F
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu

GRAD_KEYS = ("means", "scales", "quats", "opacity", "sh")


def _np(t):
    return t.detach().cpu().numpy()


def _view_tiles(vals, ranges, base, tiles_v, v, n):
    """The oracle's tile lists of view v with view-local record indices."""
    r = ranges[base:base + tiles_v].astype(np.int64)
    full = r[:, 1] > r[:, 0]
    if not full.any():
        return np.zeros(1, np.uint32), np.zeros((tiles_v, 2), np.uint32)
    lo, hi = r[full, 0].min(), r[full, 1].max()
    loc = np.where(full[:, None], r - lo, 0).astype(np.uint32)
    return (vals[lo:hi].astype(np.int64) - v * n).astype(np.uint32), loc


def _box_pixels(P):
    xs = np.arange(int(P[F["XLO"]]), int(P[F["XHI"]]) + 1)
    ys = np.arange(int(P[F["YLO"]]), int(P[F["YHI"]]) + 1)
    gx, gy = np.meshgrid(xs, ys)
    return np.stack([gx.ravel(), gy.ravel()], 1).astype(np.int32)


def _sample_records(proj, active, tiles, g, n_small, n_mid, n_large, n_heavy):
    """Visible (and active) records: small boxes (<= 64 px), larger boxes,
    the 200 largest boxes, and records of the longest tile lists."""
    ok = (proj[:, F["VALID"]] == 1) & (proj[:, F["TILES"]] > 0)
    if active is not None:
        ok &= active == 1
    area = (proj[:, F["XHI"]] - proj[:, F["XLO"]] + 1) * (proj[:, F["YHI"]] - proj[:, F["YLO"]] + 1)
    small = np.nonzero(ok & (area <= 64))[0]
    mid = np.nonzero(ok & (area > 64))[0]
    big = mid[np.argsort(area[mid])[::-1][:200]]
    vals, rng = tiles
    lens = rng[:, 1].astype(np.int64) - rng[:, 0]
    heavy_tiles = np.argsort(lens)[::-1][:8]
    heavy = np.unique(np.concatenate([vals[rng[t, 0]:rng[t, 1]] for t in heavy_tiles]).astype(np.int64))
    heavy = heavy[ok[heavy]]
    pick = []
    for pool, k in ((small, n_small), (mid, n_mid), (big, n_large), (heavy, n_heavy)):
        pool = np.setdiff1d(pool, np.array(pick, dtype=np.int64))
        pick.extend(g.choice(pool, size=min(k, pool.size), replace=False).tolist())
    return np.array(pick, dtype=np.int64), area


def _check_records(what, picks, p, cam, proj, ordr, opts, tiles, frame, pix_base, acc, acc_base, g2d_np, g2d_base,
                   dldc, n, grads=None):
    """Per sampled record: every pixel of its box against the oracle (tiled),
    its sums under the matched branches, its 2D gradient and (one view) its
    parameter gradient.  Gradients compared stacked over the sample."""
    g2_rows, o2_rows, gp_rows, op_rows = [], [], [], []
    n_amb = 0
    for i in picks:
        box = _box_pixels(proj[i])
        gidx = pix_base + box[:, 1] * cam.width + box[:, 0]
        orc = oracle.render(p, cam, proj, ordr, opts, pixels=box, tiles=tiles, accumulate=False)
        flips, na = H.match_pixels(H.gpu_pixels(frame, gidx), orc, p, cam, proj, ordr, opts, box,
                                   f"{what} record {i}", tiles=tiles)
        n_amb += na
        accr = {k: v[acc_base:acc_base + n] for k, v in acc.items()}
        H.check_accum(accr, p, cam, proj, ordr, opts, flips, n, f"{what} record {i}", pixels=box, rows=[i],
                      tiles=tiles)
        og2 = oracle.render_backward(p, cam, proj, ordr, opts, dldc[:, gidx].T.astype(np.float64), pixels=box,
                                     amb=H.AMB, flips=flips, tiles=tiles)
        o2_rows.append(og2[i])
        g2_rows.append(g2d_np[g2d_base + i].astype(np.float64))
        if grads is not None:
            sub = oracle.Params(p.means[:, [i]].copy(), p.scales[:, [i]].copy(), p.quats[:, [i]].copy(),
                                p.opacity[[i]].copy(), p.sh[:, :, [i]].copy(), p.sh_degree)
            gs = oracle.project_backward(sub, cam, opts, proj[[i]], og2[[i]])
            op_rows.append(np.concatenate([gs[k].reshape(-1) for k in GRAD_KEYS]))
            gp_rows.append(np.concatenate([grads[k][..., i].reshape(-1).astype(np.float64) for k in GRAD_KEYS]))
    e2 = H.rel_l2(np.array(g2_rows), np.array(o2_rows))
    per = [H.rel_l2(a, b) for a, b in zip(g2_rows, o2_rows)]
    H.report(what + " records", records=len(picks), box_ambiguous=n_amb, grad2d_rel_l2=e2,
             grad2d_rel_l2_median=float(np.median(per)), grad2d_rel_l2_max=float(np.max(per)))
    assert e2 <= H.GRAD_REL_L2, (what, e2)
    if grads is not None:
        ep = H.rel_l2(np.array(gp_rows), np.array(op_rows))
        H.report(what + " records params", grad_rel_l2=ep)
        assert ep <= H.GRAD_REL_L2, (what, ep)


@pytest.mark.parametrize("which", ["large", "training"])
def test_full_size_sampled_parity(gpu_lib, which):
    R = H.raster()
    wl = gs_inputs.large_scene() if which == "large" else gs_inputs.training_view()
    if wl.active is None:
        wl.active = gs_inputs.bernoulli_mask(wl.scene.n, 0.25, 2001)
    cam = wl.cameras[0]
    n, P = wl.scene.n, cam.width * cam.height
    out = H.run_gpu_forward(wl.scene, wl.cameras, accumulate=True, want_keys=True)
    dldc = gs_inputs.normal_image(3, P, 909, scale=1.0 / P)
    grads, g2d = R.render_backward(out["scene"], out["proj"], out["binned"], wl.cameras, R.RasterOpts(),
                                   out["frame"], torch.from_numpy(dldc).cuda(), torch.from_numpy(wl.active).cuda())
    torch.cuda.synchronize()
    p = oracle.Params.of(wl.scene)
    opts = oracle.Opts()
    proj = oracle.project(p, cam, opts)
    ordr = oracle.order(proj)
    # binning, bit-exact in full
    tx, ty, base, total = oracle.view_layout(wl.cameras)
    keys, vals, ranges = oracle.bin(oracle.tile_rects(proj), oracle.zbits(proj), 1, n, base, tx, total)
    b = out["binned"]
    assert b.stats.n_isect == len(keys)
    assert np.array_equal(_np(b.keys).view(np.uint64), keys)
    assert np.array_equal(_np(b.vals).view(np.uint32), vals)
    assert np.array_equal(_np(b.ranges).view(np.uint32), ranges)
    H.check_bin_extras(b, oracle.tile_rects(proj), oracle.zbits(proj), 1, total, ranges, which)
    del keys
    # sampled pixels, every one checked: 64 over every Gaussian (untiled, so the
    # tiling itself is under test) and 2000 over their tile's list
    g = gs_inputs.rng(17)
    fr = out["frame"]
    tiles = _view_tiles(vals, ranges, 0, total, 0, n)
    for m, tl in ((64, None), (2000, tiles)):
        pix = np.stack([g.integers(0, cam.width, m), g.integers(0, cam.height, m)], 1).astype(np.int32)
        orc = oracle.render(p, cam, proj, ordr, opts, pixels=pix, tiles=tl, accumulate=False)
        idx = pix[:, 1] * cam.width + pix[:, 0]
        _, namb = H.match_pixels(H.gpu_pixels(fr, idx), orc, p, cam, proj, ordr, opts, pix,
                                 f"{which} sampled pixels", tiles=tl)
        H.report(f"{which} sampled pixels ({'tiled' if tl else 'untiled'})", pixels=m, ambiguous=namb)
        assert (orc["imax"] >= 0).sum() > m // 10  # the sample does hit the scene (~20% coverage at radius 30)
    # 50 sampled Gaussians: every pixel of their box, their sums and gradients
    picks, area = _sample_records(proj, wl.active, tiles, g, 15, 15, 10, 10)
    assert len(picks) == 50 and area[picks].max() > 256
    acc = {k: _np(v) for k, v in out["acc"].items()}
    gnp = {k: _np(v) for k, v in grads.items()}
    _check_records(which, picks, p, cam, proj, ordr, opts, tiles, fr, 0, acc, 0, _np(g2d), 0, dldc, n, gnp)
    # invariants over the whole image
    imp = acc["importance"].astype(np.float64)
    tf = _np(fr.t_final).astype(np.float64)
    assert imp.sum() == pytest.approx((1 - tf).sum(), rel=1e-4)
    assert int(acc["area"].sum()) == int((_np(fr.imax) >= 0).sum())
    assert np.all(acc["wmax"] <= np.minimum(acc["importance"], 0.99) + 1e-6)
    # inactive Gaussians receive exactly zero
    ina = wl.active == 0
    for k in GRAD_KEYS:
        assert np.all(gnp[k][..., ina] == 0)


def test_multiview_full_size_sampled_parity(gpu_lib):
    """1M Gaussians, 16 views of mixed resolution in one launch per stage: the
    binning bit-exact in full, sampled pixels of three views over every
    Gaussian, per-view sums and 2D gradients of 17 sampled records per view
    from every pixel of their box, and per-view invariants over every image."""
    R = H.raster()
    wl = gs_inputs.multiview()
    cams = wl.cameras
    n, V = wl.scene.n, len(cams)
    out = H.run_gpu_forward(wl.scene, cams, accumulate=True, per_view=True, want_keys=True)
    lay = R.view_layout(cams)
    P = lay.pixels_total
    dldc = gs_inputs.normal_image(3, P, 910, scale=1.0 / P)
    _, g2d = R.render_backward(out["scene"], out["proj"], out["binned"], cams, R.RasterOpts(), out["frame"],
                               torch.from_numpy(dldc).cuda())
    torch.cuda.synchronize()
    p = oracle.Params.of(wl.scene)
    opts = oracle.Opts()
    projs = [oracle.project(p, c, opts) for c in cams]
    # binning of all views, bit-exact in full (records of view v are v * n + i)
    tx, ty, base, total = oracle.view_layout(cams)
    rects = np.concatenate([oracle.tile_rects(q) for q in projs])
    zb = np.concatenate([oracle.zbits(q) for q in projs])
    keys, vals, ranges = oracle.bin(rects, zb, V, n, base, tx, total)
    b = out["binned"]
    assert b.stats.n_isect == len(keys) > 10 ** 7
    assert np.array_equal(_np(b.keys).view(np.uint64), keys)
    assert np.array_equal(_np(b.vals).view(np.uint32), vals)
    assert np.array_equal(_np(b.ranges).view(np.uint32), ranges)
    H.check_bin_extras(b, rects, zb, V, total, ranges, f"{V} views")
    del rects, zb
    del keys
    fr = out["frame"]
    acc = {k: _np(t) for k, t in out["acc"].items()}
    imax_all, tf_all = _np(fr.imax), _np(fr.t_final).astype(np.float64)
    g2d_np = _np(g2d)
    g = gs_inputs.rng(19)
    for v in (0, 9, 15):
        cam, proj = cams[v], projs[v]
        ordr = oracle.order(proj)
        pb = lay.pixel_base[v]
        tiles = _view_tiles(vals, ranges, int(base[v]), int(tx[v] * ty[v]), v, n)
        for m, tl in ((48, None), (1000, tiles)):
            pix = np.stack([g.integers(0, cam.width, m), g.integers(0, cam.height, m)], 1).astype(np.int32)
            orc = oracle.render(p, cam, proj, ordr, opts, pixels=pix, tiles=tl, accumulate=False)
            idx = pb + pix[:, 1] * cam.width + pix[:, 0]
            _, namb = H.match_pixels(H.gpu_pixels(fr, idx), orc, p, cam, proj, ordr, opts, pix, f"view {v} pixels",
                                     tiles=tl)
            H.report(f"multiview view {v} sampled pixels ({'tiled' if tl else 'untiled'})", pixels=m, ambiguous=namb)
            assert (orc["imax"] >= 0).sum() > m // 2, v  # radius 6 around the scene: most pixels are covered
        picks, _ = _sample_records(proj, None, tiles, g, 5, 5, 4, 3)
        assert len(picks) == 17, v
        _check_records(f"multiview view {v}", picks, p, cam, proj, ordr, opts, tiles, fr, pb, acc, v * n, g2d_np,
                       v * n, dldc, n)
    # per-view invariants over every image
    for v, cam in enumerate(cams):
        sl = slice(lay.pixel_base[v], lay.pixel_base[v] + cam.width * cam.height)
        rows = slice(v * n, (v + 1) * n)
        assert acc["importance"][rows].astype(np.float64).sum() == pytest.approx((1 - tf_all[sl]).sum(), rel=1e-4)
        assert int(acc["area"][rows].sum()) == int((imax_all[sl] >= 0).sum())
