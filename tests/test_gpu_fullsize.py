"""Parity at full workload sizes, in the launch configuration the benchmark
times: 3M Gaussians at 1920x1080 and 500k at 1245x825.  The oracle computes
sampled outputs one by one (pixels over every Gaussian; per-Gaussian gradients
and sums from the pixels of that Gaussian's box) and the binning in full."""
import numpy as np
import pytest
import torch

import gs_inputs
import oracle
from oracle import F
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


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
    # sampled pixels over every Gaussian
    g = gs_inputs.rng(17)
    m = 300
    pix = np.stack([g.integers(0, cam.width, m), g.integers(0, cam.height, m)], 1).astype(np.int32)
    orc = oracle.render(p, cam, proj, ordr, opts, pixels=pix, accumulate=False)
    idx = pix[:, 1] * cam.width + pix[:, 0]
    fr = out["frame"]
    amb = H.ambiguous(orc)
    amb_arg = H.ambiguous(orc, argmax=True)
    assert amb_arg.sum() <= 3
    col = _np(fr.color[:, torch.from_numpy(idx).cuda()]).T.astype(np.float64)
    assert np.abs(col - orc["color"])[~amb].max() <= H.COLOR_ATOL
    assert np.abs(_np(fr.t_final)[idx] - orc["t_final"])[~amb].max() <= H.COLOR_ATOL
    assert np.array_equal(_np(fr.n_contrib)[idx][~amb], orc["n_contrib"][~amb])
    assert np.array_equal(_np(fr.imax)[idx][~amb_arg], orc["imax"][~amb_arg])
    assert np.abs(_np(fr.depth)[idx] - orc["depth"])[~amb_arg].max() <= H.COLOR_ATOL
    assert (orc["imax"] >= 0).sum() > m // 10  # the sample does hit the scene (~20% coverage at radius 30)
    # sampled Gaussians: 2D gradient, parameter gradient and sums from the pixels of their box
    vis = np.nonzero((proj[:, F["VALID"]] == 1) & (proj[:, F["TILES"]] > 0) & (wl.active == 1) &
                     ((proj[:, F["XHI"]] - proj[:, F["XLO"]] + 1) * (proj[:, F["YHI"]] - proj[:, F["YLO"]] + 1)
                      <= 64))[0]
    pick = g.choice(vis, size=24, replace=False)
    g2_rows, o2_rows, gp_rows, op_rows = [], [], [], []
    g2d_np = _np(g2d)
    acc = {k: _np(v) for k, v in out["acc"].items()}
    for i in pick:
        if len(o2_rows) >= 10:
            break
        P_ = proj[i]
        xs = np.arange(int(P_[F["XLO"]]), int(P_[F["XHI"]]) + 1)
        ys = np.arange(int(P_[F["YLO"]]), int(P_[F["YHI"]]) + 1)
        box = np.array([(x, y) for y in ys for x in xs], dtype=np.int32)
        bidx = box[:, 1] * cam.width + box[:, 0]
        r_orc = oracle.render(p, cam, proj, ordr, opts, pixels=box, accumulate=True)
        if H.ambiguous(r_orc, argmax=True).any():
            continue
        og2 = oracle.render_backward(p, cam, proj, ordr, opts, dldc[:, bidx].T.astype(np.float64), pixels=box)
        o2_rows.append(og2[i])
        g2_rows.append(g2d_np[i].astype(np.float64))
        sub = p.copy()
        sub = oracle.Params(sub.means[:, [i]].copy(), sub.scales[:, [i]].copy(), sub.quats[:, [i]].copy(),
                            sub.opacity[[i]].copy(), sub.sh[:, :, [i]].copy(), sub.sh_degree)
        gs = oracle.project_backward(sub, cam, opts, proj[[i]], og2[[i]])
        op_rows.append(np.concatenate([gs[k].reshape(-1) for k in ("means", "scales", "quats", "opacity", "sh")]))
        gp_rows.append(np.concatenate([_np(grads[k])[..., i].reshape(-1).astype(np.float64)
                                       for k in ("means", "scales", "quats", "opacity", "sh")]))
        assert acc["importance"][i] == pytest.approx(r_orc["importance"][i], rel=1e-4, abs=1e-6)
        assert acc["wmax"][i] == pytest.approx(r_orc["wmax"][i], rel=1e-5, abs=1e-7)
        assert acc["area"][i] == r_orc["area"][i]
    assert len(o2_rows) >= 6
    assert H.rel_l2(np.array(g2_rows), np.array(o2_rows)) <= H.GRAD_REL_L2
    assert H.rel_l2(np.array(gp_rows), np.array(op_rows)) <= H.GRAD_REL_L2
    # invariants over the whole image
    imp = acc["importance"].astype(np.float64)
    tf = _np(fr.t_final).astype(np.float64)
    assert imp.sum() == pytest.approx((1 - tf).sum(), rel=1e-4)
    assert int(acc["area"].sum()) == int((_np(fr.imax) >= 0).sum())
    assert np.all(acc["wmax"] <= np.minimum(acc["importance"], 0.99) + 1e-6)
    # inactive Gaussians receive exactly zero
    ina = wl.active == 0
    for k in ("means", "opacity"):
        assert np.all(_np(grads[k])[..., ina] == 0)


def test_multiview_full_size_sampled_parity(gpu_lib):
    """1M Gaussians, 16 views of mixed resolution in one launch per stage: the
    binning bit-exact in full, sampled pixels of three views over every
    Gaussian, per-view sums and 2D gradients of sampled records from the pixels
    of their box, and per-view invariants over every image."""
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
    tx, _, base, total = oracle.view_layout(cams)
    keys, vals, ranges = oracle.bin(np.concatenate([oracle.tile_rects(q) for q in projs]),
                                    np.concatenate([oracle.zbits(q) for q in projs]), V, n, base, tx, total)
    b = out["binned"]
    assert b.stats.n_isect == len(keys) > 10 ** 7
    assert np.array_equal(_np(b.keys).view(np.uint64), keys)
    assert np.array_equal(_np(b.vals).view(np.uint32), vals)
    assert np.array_equal(_np(b.ranges).view(np.uint32), ranges)
    del keys, vals
    fr = out["frame"]
    acc = {k: _np(t) for k, t in out["acc"].items()}
    imax_all, tf_all = _np(fr.imax), _np(fr.t_final).astype(np.float64)
    g2d_np = _np(g2d)
    g = gs_inputs.rng(19)
    for v in (0, 9, 15):
        cam, proj = cams[v], projs[v]
        ordr = oracle.order(proj)
        pb = lay.pixel_base[v]
        m = 100
        pix = np.stack([g.integers(0, cam.width, m), g.integers(0, cam.height, m)], 1).astype(np.int32)
        orc = oracle.render(p, cam, proj, ordr, opts, pixels=pix, accumulate=False)
        idx = pb + pix[:, 1] * cam.width + pix[:, 0]
        amb, amb_arg = H.ambiguous(orc), H.ambiguous(orc, argmax=True)
        assert amb_arg.sum() <= 10, v  # dense views: a few pixels sit near an argmax tie
        col = _np(fr.color[:, torch.from_numpy(idx).cuda()]).T.astype(np.float64)
        assert np.abs(col - orc["color"])[~amb].max() <= H.COLOR_ATOL, v
        assert np.abs(tf_all[idx] - orc["t_final"])[~amb].max() <= H.COLOR_ATOL, v
        assert np.array_equal(_np(fr.n_contrib)[idx][~amb], orc["n_contrib"][~amb]), v
        assert np.array_equal(imax_all[idx][~amb_arg], orc["imax"][~amb_arg]), v
        assert np.abs(_np(fr.depth)[idx] - orc["depth"])[~amb_arg].max() <= H.COLOR_ATOL, v
        assert (orc["imax"] >= 0).sum() > m // 2, v  # radius 6 around the scene: most pixels are covered
        # sampled records of this view: per-view sums and the 2D gradient
        vis = np.nonzero((proj[:, F["VALID"]] == 1) & (proj[:, F["TILES"]] > 0) &
                         ((proj[:, F["XHI"]] - proj[:, F["XLO"]] + 1) * (proj[:, F["YHI"]] - proj[:, F["YLO"]] + 1)
                          <= 64))[0]
        g2_rows, o2_rows = [], []
        for i in g.choice(vis, size=16, replace=False):
            if len(o2_rows) >= 4:
                break
            xs = np.arange(int(proj[i, F["XLO"]]), int(proj[i, F["XHI"]]) + 1)
            ys = np.arange(int(proj[i, F["YLO"]]), int(proj[i, F["YHI"]]) + 1)
            box = np.array([(x, y) for y in ys for x in xs], dtype=np.int32)
            r_orc = oracle.render(p, cam, proj, ordr, opts, pixels=box, accumulate=True)
            if H.ambiguous(r_orc, argmax=True).any():
                continue
            bidx = pb + box[:, 1] * cam.width + box[:, 0]
            og2 = oracle.render_backward(p, cam, proj, ordr, opts, dldc[:, bidx].T.astype(np.float64), pixels=box)
            o2_rows.append(og2[i])
            g2_rows.append(g2d_np[v * n + i].astype(np.float64))
            assert acc["importance"][v * n + i] == pytest.approx(r_orc["importance"][i], rel=1e-4, abs=1e-6)
            assert acc["wmax"][v * n + i] == pytest.approx(r_orc["wmax"][i], rel=1e-5, abs=1e-7)
            assert acc["area"][v * n + i] == r_orc["area"][i]
        assert len(o2_rows) >= 3, v
        assert H.rel_l2(np.array(g2_rows), np.array(o2_rows)) <= H.GRAD_REL_L2, v
    # per-view invariants over every image
    for v, cam in enumerate(cams):
        sl = slice(lay.pixel_base[v], lay.pixel_base[v] + cam.width * cam.height)
        rows = slice(v * n, (v + 1) * n)
        assert acc["importance"][rows].astype(np.float64).sum() == pytest.approx((1 - tf_all[sl]).sum(), rel=1e-4)
        assert int(acc["area"][rows].sum()) == int((imax_all[sl] >= 0).sum())
