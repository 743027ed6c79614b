"""Differentiation pattern: torch.autograd.Function with recompute-in-backward,
batched multi-view launches, gradients vs the FP64 oracle (analytic and
central finite differences on a 256-Gaussian subset)."""
import numpy as np
import pytest
import torch

import gs_inputs
import oracle
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda().float().requires_grad_(True)


def _leaves(sc):
    return [_t(sc.means), _t(sc.scales), _t(sc.quats), _t(sc.opacity), _t(sc.sh)]


def _cams():
    res = [(64, 48), (80, 60), (96, 72), (48, 48)]
    return gs_inputs.sphere_cameras(4, 3.0, res, 31)


def _scene256():
    return gs_inputs.surface_scene(256, 17, centre_half=0.6, log_scale_mu=-2.6, log_scale_sd=0.3)


def _run(leaves, cams, g, **kw):
    from paper_2411_12788_amd.autograd import rasterize
    color, depth, imax = rasterize(*leaves, cams, **kw)
    (color * g).sum().backward()
    return color, [x.grad.detach().clone() for x in leaves]


def test_recompute_matches_saved_lists_and_direct_backward(gpu_lib):
    R = H.raster()
    sc = _scene256()
    cams = _cams()
    lay = R.view_layout(cams)
    g = torch.from_numpy(gs_inputs.normal_image(3, lay.pixels_total, 3, 1e-3)).cuda()
    col_a, ga = _run(_leaves(sc), cams, g)
    col_b, gb = _run(_leaves(sc), cams, g, save_lists=True)
    assert torch.equal(col_a, col_b)
    for x, y in zip(ga, gb):
        # float atomics may add in a different order; the lists themselves are
        # identical.  A reordered float32 sum differs by a few ulps of its
        # running magnitude, which the largest entry of the group bounds.
        assert float((x - y).abs().max()) <= 1e-5 * float(x.abs().max()) + 1e-12
    ds = R.DeviceScene.from_numpy(sc)
    p1 = R.project(ds, cams, R.RasterOpts())
    b1 = R.bin(p1, cams, ds.n)
    p2 = R.project(ds, cams, R.RasterOpts())
    b2 = R.bin(p2, cams, ds.n)
    drawn = p1.bin.view(-1, 4)[:, 3] > 0  # the records the library writes
    assert torch.equal(p1.bin, p2.bin) and bool(drawn.any())
    assert torch.equal(p1.rec.view(-1, 16)[drawn], p2.rec.view(-1, 16)[drawn])
    assert torch.equal(b1.vals, b2.vals) and torch.equal(b1.ranges, b2.ranges)


def test_batched_views_equal_sum_of_single_views(gpu_lib):
    R = H.raster()
    sc = _scene256()
    cams = _cams()
    lay = R.view_layout(cams)
    g = torch.from_numpy(gs_inputs.normal_image(3, lay.pixels_total, 4, 1e-3)).cuda()
    col, gb = _run(_leaves(sc), cams, g)
    tot = None
    for v, cam in enumerate(cams):
        sl = slice(lay.pixel_base[v], lay.pixel_base[v] + cam.width * cam.height)
        c1, g1 = _run(_leaves(sc), [cam], g[:, sl].contiguous())
        assert torch.equal(c1, col[:, sl])
        tot = g1 if tot is None else [a + b for a, b in zip(tot, g1)]
    for x, y in zip(gb, tot):
        # same sums, grouped per view instead of over all views at once
        assert float((x - y).abs().max()) <= 1e-4 * float(x.abs().max()) + 1e-12


def test_gradients_vs_oracle_and_finite_differences_256(gpu_lib):
    R = H.raster()
    sc = _scene256()
    cams = _cams()
    lay = R.view_layout(cams)
    gnp = gs_inputs.normal_image(3, lay.pixels_total, 5, 1e-3)
    g = torch.from_numpy(gnp).cuda()
    _, grads = _run(_leaves(sc), cams, g)
    names = ["means", "scales", "quats", "opacity", "sh"]
    gg = {k: v.double().cpu().numpy() for k, v in zip(names, grads)}
    p = oracle.Params.of(sc)
    opts = oracle.Opts()
    dl = [gnp[:, lay.pixel_base[v]:lay.pixel_base[v] + c.width * c.height].T.astype(np.float64)
          for v, c in enumerate(cams)]
    og, _ = oracle.backward_views(p, cams, opts, dl)
    for k in names:
        assert H.rel_l2(gg[k], og[k]) <= H.GRAD_REL_L2, k

    def loss(pp):
        s = 0.0
        for v, c in enumerate(cams):
            s += float((oracle.forward_view(pp, c, opts, accumulate=False)["color"] * dl[v]).sum())
        return s

    margins = [oracle.forward_view(p, c, opts, accumulate=False)["margin"] for c in cams]
    mmin = min(min(m[:, 0].min(), m[:, 1].min()) for m in margins)
    # a 1e-7 relative perturbation moves alpha by <= ~1e-6 relative: decisions need a larger margin
    assert mmin > 2e-6, mmin
    rng = gs_inputs.rng(6)
    fd_vals, gpu_vals, an_vals = [], [], []
    for _ in range(120):
        k = names[int(rng.integers(0, len(names)))]
        arr = getattr(p, k)
        idx = tuple(int(rng.integers(0, s)) for s in arr.shape)
        if k == "sh" and idx[0] >= 16:
            continue
        x0 = arr[idx]
        h = 1e-7 * max(1.0, abs(x0))
        pa, pb = p.copy(), p.copy()
        getattr(pa, k)[idx] = x0 + h
        getattr(pb, k)[idx] = x0 - h
        fd_vals.append((loss(pa) - loss(pb)) / (2 * h))
        gpu_vals.append(gg[k][idx])
        an_vals.append(og[k][idx])
    fd_vals, gpu_vals, an_vals = map(np.array, (fd_vals, gpu_vals, an_vals))
    assert H.rel_l2(an_vals, fd_vals) <= 1e-5
    assert H.rel_l2(gpu_vals, fd_vals) <= H.GRAD_REL_L2
