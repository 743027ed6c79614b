"""Deterministic gradient reduction (ordered, atomic-free), through the C ABI:
bitwise the same from run to run, equal to the float-atomic path up to
float32 summation order, parity with the FP64 oracle, zero rows for inactive
Gaussians, and the autograd wrapper's two modes bitwise equal with it.  Also
the tile processing order: a stable function of the ranges."""
import numpy as np
import pytest
import torch

import gs_inputs
import oracle
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _backward(out, cams, dldc, active, deterministic, R):
    grads, g2d = R.render_backward(out["scene"], out["proj"], out["binned"], cams, R.RasterOpts(), out["frame"],
                                   dldc, active, deterministic=deterministic)
    torch.cuda.synchronize()
    return {k: v.clone() for k, v in grads.items()}, g2d.clone()


CASES = {
    "small cube": lambda: gs_inputs.small_cube(seed=5, n=3000, width=112, height=96),
    # every tile long: the split work items (four workgroups per tile)
    "heavy tiles": lambda: gs_inputs.heavy_tiles(seed=7, opacity=(0.05, 0.3)),
    "concentrated": lambda: gs_inputs.heavy_tiles(seed=9, n=20_000, width=128, height=96, opacity=(0.02, 0.2),
                                                  distance=9.0),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("masked", [False, True])
def test_deterministic_backward(gpu_lib, case, masked):
    R = H.raster()
    wl = CASES[case]()
    cam = wl.cameras[0]
    n, Pn = wl.scene.n, cam.width * cam.height
    print(f"deterministic backward: {case}, masked={masked}, n={n}", flush=True)
    out = H.run_gpu_forward(wl.scene, wl.cameras, accumulate=False)
    dldc = torch.from_numpy(gs_inputs.normal_image(3, Pn, 51, scale=1.0 / Pn)).cuda()
    active = torch.from_numpy(gs_inputs.bernoulli_mask(n, 0.25, 52)).cuda() if masked else None
    g1, d1 = _backward(out, wl.cameras, dldc, active, True, R)
    g2, d2 = _backward(out, wl.cameras, dldc, active, True, R)
    ga, da = _backward(out, wl.cameras, dldc, active, False, R)
    # bitwise the same from run to run
    assert torch.equal(d1, d2)
    for k in g1:
        assert torch.equal(g1[k], g2[k]), k
    # the atomic path sums the same terms in another order
    assert H.rel_l2(_np(d1), _np(da)) <= 1e-5
    for k in g1:
        assert H.rel_l2(_np(g1[k]), _np(ga[k])) <= 1e-5, k
    if masked:
        ina = _np(active) == 0
        assert np.all(_np(d1)[:n][ina] == 0)
        for k in g1:
            assert np.all(_np(g1[k])[..., :n][..., ina] == 0), k
    # parity with the oracle under the branches the forward took
    p = oracle.Params.of(wl.scene)
    orc = oracle.forward_view(p, cam, oracle.Opts())
    flips, _ = H.compare_forward(out["frame"], orc, slice(0, Pn), f"det {case}", p, cam)
    og, _ = H.backward_views(p, wl.cameras, oracle.Opts(), [_np(dldc).T.astype(np.float64)],
                             active=None if active is None else _np(active), flips=[flips])
    for k in ("means", "scales", "quats", "opacity", "sh"):
        assert H.rel_l2(_np(g1[k]).astype(np.float64)[..., :n], og[k]) <= H.GRAD_REL_L2, k


def test_deterministic_backward_multiview_and_tile_culling(gpu_lib):
    """Several views in one launch, and tile culling at emission (pairs are
    ranked among the kept tiles of their record)."""
    R = H.raster()
    sc = gs_inputs.uniform_cube_scene(2500, 9)
    cams = [gs_inputs.look_at((0, 0, 4), (0, 0, 0), 96, 64), gs_inputs.look_at((2.5, 1, 3), (0, 0, 0), 50, 37),
            gs_inputs.look_at((-3, 0.5, 2.5), (0, 0, 0), 128, 80)]
    lay = R.view_layout(cams)
    dldc = torch.from_numpy(gs_inputs.normal_image(3, lay.pixels_total, 61, scale=1e-3)).cuda()
    p = oracle.Params.of(sc)
    results = []
    for cull in (False, True):
        out = H.run_gpu_forward(sc, cams, opts=R.RasterOpts(tile_cull=cull), accumulate=False)
        g1, d1 = _backward(out, cams, dldc, None, True, R)
        g2, d2 = _backward(out, cams, dldc, None, True, R)
        assert torch.equal(d1, d2)
        fls = []
        for v, cam in enumerate(cams):
            orc = oracle.forward_view(p, cam, oracle.Opts())
            sl = slice(lay.pixel_base[v], lay.pixel_base[v] + cam.width * cam.height)
            flips, _ = H.compare_forward(out["frame"], orc, sl, f"det view {v} cull {cull}", p, cam)
            fls.append(flips)
        per_view = [_np(dldc)[:, lay.pixel_base[v]:lay.pixel_base[v] + c.width * c.height].T.astype(np.float64)
                    for v, c in enumerate(cams)]
        og, _ = H.backward_views(p, cams, oracle.Opts(), per_view, flips=fls)
        for k in og:
            assert H.rel_l2(_np(g1[k]).astype(np.float64)[..., :sc.n], og[k]) <= H.GRAD_REL_L2, (k, cull)
        results.append(g1)
    # dropped pairs could never composite: the gradients agree
    for k in results[0]:
        assert H.rel_l2(_np(results[1][k]), _np(results[0][k])) <= 1e-5, k


def test_autograd_modes_bitwise_equal_with_deterministic_reduction(gpu_lib):
    from paper_2411_12788_amd.autograd import rasterize
    R = H.raster()
    sc = gs_inputs.surface_scene(40_000, 71)
    cams = [gs_inputs.look_at((0, 0, 6), (0, 0, 0), 160, 120), gs_inputs.look_at((4, 2, 4), (0, 0, 0), 128, 96)]
    ds = R.DeviceScene.from_numpy(sc)
    lay = R.view_layout(cams)
    target = torch.from_numpy(gs_inputs.uniform_image(3, lay.pixels_total, 72)).cuda()
    got = []
    for save_lists in (False, True, False):
        leaves = [t.clone().requires_grad_(True) for t in (ds.means, ds.scales, ds.quats, ds.opacity, ds.sh)]
        color, _, _ = rasterize(*leaves, cams, save_lists=save_lists, deterministic=True)
        (color - target).abs().mean().backward()
        torch.cuda.synchronize()
        got.append([x.grad.clone() for x in leaves])
    for a, b in zip(got[0], got[1]):
        assert torch.equal(a, b)
    for a, b in zip(got[0], got[2]):
        assert torch.equal(a, b)


def test_tile_order_is_stable(gpu_lib):
    """Longest lists first, ascending tile id inside each bit-length group, and
    the same order from run to run."""
    R = H.raster()
    wl = gs_inputs.small_cube(seed=6)
    out = H.run_gpu_forward(wl.scene, wl.cameras, accumulate=False)
    b = out["binned"]
    order = _np(b.order).astype(np.int64)
    rng = _np(b.ranges).view(np.uint32).astype(np.int64)
    L = rng[:, 1] - rng[:, 0]
    bits = np.array([int(x).bit_length() for x in L])
    want = np.lexsort((np.arange(len(L)), -bits))
    assert np.array_equal(order, want)
    out2 = H.run_gpu_forward(wl.scene, wl.cameras, accumulate=False)
    assert torch.equal(out2["binned"].order, b.order)
