"""GPU parity of the culling and densification criteria against the oracle
(Sec. 5.1, Sec. 5.2, Eq. (3)) on seeded synthetic accumulations.

The value-mode threshold is an order statistic: tau and the masks must match
bit for bit.  The mass-mode threshold compares prefix sums whose rounding
depends on summation order; a case is exempt only when the oracle reports a
decision margin below the FP64 summation error bound 8 m 2^-53 S.
"""
import math

import numpy as np
import pytest
import torch

import gs_inputs
import oracle

pytestmark = pytest.mark.gpu

VALUE, MASS = oracle.THRESHOLD_VALUE, oracle.THRESHOLD_MASS


def D():
    from paper_2411_12788_amd import densify
    return densify


def _ambiguous(margin, values):
    v = np.asarray(values, dtype=np.float64)
    v = v[v > 0]
    return margin < 8.0 * max(v.shape[0], 1) * 2.0 ** -53 * float(v.sum())


def _check_visibility(imp, keep, mode):
    V, n = imp.shape
    vis_g, tau_g = D().visibility(torch.from_numpy(imp).cuda(), keep, mode)
    vis_g, tau_g = vis_g.cpu().numpy(), tau_g.cpu().numpy()
    for k in range(V):
        vis_o, tau_o, margin = oracle.visibility(imp[k], keep, mode)
        if mode == MASS and _ambiguous(margin, imp[k]):
            continue
        if math.isnan(tau_o):
            assert math.isnan(tau_g[k]) and not vis_g[k].any()
            continue
        assert tau_g[k] == tau_o, (k, tau_g[k], tau_o)
        assert (vis_g[k] == vis_o).all(), (k, int((vis_g[k] != vis_o).sum()))


@pytest.mark.parametrize("mode", [VALUE, MASS])
@pytest.mark.parametrize("seed,V,n", [(0, 1, 1), (1, 1, 1000), (2, 4, 50_000), (3, 3, 4097), (4, 2, 200_003)])
def test_visibility_matches_oracle(gpu_lib, mode, seed, V, n):
    _check_visibility(gs_inputs.importance_like(V, n, seed), 0.99, mode)


@pytest.mark.parametrize("mode", [VALUE, MASS])
@pytest.mark.parametrize("keep", [0.0, 0.5, 0.9, 1.0])
def test_visibility_keep_values(gpu_lib, mode, keep):
    _check_visibility(gs_inputs.importance_like(2, 30_000, 11), keep, mode)


@pytest.mark.parametrize("mode", [VALUE, MASS])
def test_visibility_degenerate(gpu_lib, mode):
    # no contributor, one contributor, all equal, two distinct values, a few huge values
    cases = [np.zeros(100), np.eye(1, 100, 37)[0] * 3.0, np.full(777, 0.25),
             np.r_[np.full(500, 0.5), np.full(500, 2.0)], np.r_[np.full(10_000, 1e-3), np.full(3, 1e6)]]
    for c in cases:
        _check_visibility(c.astype(np.float32)[None, :], 0.99, mode)


def test_visibility_empty(gpu_lib):
    vis, tau = D().visibility(torch.zeros((3, 0), device="cuda"))
    assert vis.shape == (3, 0) and torch.isnan(tau).all()


@pytest.mark.parametrize("mode", [VALUE, MASS])
@pytest.mark.parametrize("seed,n", [(0, 1), (1, 5000), (2, 333_333)])
def test_critical_matches_oracle(gpu_lib, mode, seed, n):
    area, wmax = gs_inputs.wmax_like(n, seed)
    crit_g, tau_g = D().critical(torch.from_numpy(area.view(np.int32)).cuda(), torch.from_numpy(wmax).cuda(), 0.99,
                                 mode)
    crit_o, tau_o, margin = oracle.critical(area, wmax, 0.99, mode)
    if mode == MASS and _ambiguous(margin, np.where(area > 0, wmax, 0)):
        pytest.skip("threshold decision within the summation error bound")
    tau_g = float(tau_g.cpu()[0])
    if math.isnan(tau_o):
        assert math.isnan(tau_g)
    else:
        assert tau_g == tau_o
    assert (crit_g.cpu().numpy() == crit_o).all()


@pytest.mark.parametrize("H,W", [(1080, 1920), (825, 1245), (7, 3)])
def test_blur_split_matches_oracle(gpu_lib, H, W):
    g = gs_inputs.rng(5)
    area = g.integers(0, 2 * int(2e-4 * H * W) + 3, size=100_001).astype(np.uint32)
    thr = int(2e-4 * H * W)
    area[:3] = [thr, thr + 1, 0]
    got = D().blur_split(torch.from_numpy(area.view(np.int32)).cuda(), H, W).cpu().numpy()
    assert (got == oracle.blur_split(area, H, W)).all()


def _ulp_diff(a, b):
    a = np.asarray(a, np.float32).view(np.int32).astype(np.int64)
    b = np.asarray(b, np.float32).view(np.int32).astype(np.int64)
    return np.abs(a - b)


@pytest.mark.parametrize("seed,n,frac", [(0, 1, 1.0), (1, 4096, 0.3), (2, 4097, 0.3), (3, 100_000, 0.05),
                                         (4, 20_000, 1.0), (5, 20_000, 0.0)])
def test_clone_matches_oracle(gpu_lib, seed, n, frac):
    R = __import__("paper_2411_12788_amd.raster", fromlist=["DeviceScene"])
    scene = gs_inputs.uniform_cube_scene(n, seed=seed)
    op = scene.opacity.copy()
    op[: min(n, 4)] = np.array([0.0, 1.0, 1e-7, 0.5], np.float32)[: min(n, 4)]
    scene.opacity = op
    sel = gs_inputs.bernoulli_mask(n, frac, seed + 100)
    ds = R.DeviceScene.from_numpy(scene)
    out, count = D().clone(ds, torch.from_numpy(sel).cuda())
    ref = oracle.clone(oracle.Params.of(scene), sel)
    assert int(count.cpu()[0]) == int(sel.sum()) == ref.n - n
    for name in ("means", "quats", "sh"):
        assert (getattr(out, name).cpu().numpy() == getattr(ref, name).astype(np.float32)).all(), name
    for name in ("scales", "opacity"):
        d = _ulp_diff(getattr(out, name).cpu().numpy(), getattr(ref, name).astype(np.float32))
        assert d.max() <= 1, (name, int(d.max()))
    # the two copies recompose the original peak opacity
    a = out.opacity.cpu().numpy().astype(np.float64)
    idx = np.nonzero(sel)[0]
    if idx.size:
        comp = 1 - (1 - a[idx]) ** 2
        assert np.allclose(comp, scene.opacity[idx].astype(np.float64), rtol=1e-6, atol=1e-7)


def test_clone_capacity_drops_extra_copies(gpu_lib):
    R = __import__("paper_2411_12788_amd.raster", fromlist=["DeviceScene"])
    n = 1000
    scene = gs_inputs.uniform_cube_scene(n, seed=9)
    sel = np.ones(n, np.uint8)
    ds = R.DeviceScene.from_numpy(scene)
    out, count = D().clone(ds, torch.from_numpy(sel).cuda(), capacity=n + 10)
    ref = oracle.clone(oracle.Params.of(scene), sel)
    assert int(count.cpu()[0]) == n
    assert (out.means.cpu().numpy() == ref.means[:, : n + 10].astype(np.float32)).all()


def test_grad_stats_matches_oracle(gpu_lib):
    from paper_2411_12788_amd import raster as R
    V, n = 3, 10_007
    g = gs_inputs.rng(21)
    tiles = g.integers(-1, 4, size=(V, n)).astype(np.int32)
    grad2d = gs_inputs.normal_image(V * n, 9, 22)                   # [V * n, 9]
    cams = [gs_inputs.look_at((0, 0, 4), (0, 0, 0), w, h) for (w, h) in [(640, 480), (1920, 1080), (33, 17)]]
    bin_ = np.zeros((V * n, 4), np.int32)
    bin_[:, 3] = tiles.reshape(-1)
    proj = R.Projected(torch.zeros((V * n, 16), device="cuda"), torch.from_numpy(bin_).cuda())
    ns = torch.zeros(n, device="cuda")
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    D().grad_stats(proj, torch.from_numpy(grad2d).cuda(), cams, n, ns, cnt)
    ns_o, cnt_o = oracle.grad_stats(tiles, grad2d, [c.width for c in cams], [c.height for c in cams])
    assert (cnt.cpu().numpy() == cnt_o).all()
    np.testing.assert_allclose(ns.cpu().numpy(), ns_o, rtol=2e-6, atol=1e-6)


@pytest.mark.parametrize("mode", [VALUE, MASS])
def test_thresholds_full_size(gpu_lib, mode):
    """3M Gaussians, the large-scene size: one view's visibility and the critical set."""
    imp = gs_inputs.importance_like(1, 3_000_000, 31)
    _check_visibility(imp, 0.99, mode)
    area, wmax = gs_inputs.wmax_like(3_000_000, 32)
    crit_g, tau_g = D().critical(torch.from_numpy(area.view(np.int32)).cuda(), torch.from_numpy(wmax).cuda(), 0.99,
                                 mode)
    crit_o, tau_o, margin = oracle.critical(area, wmax, 0.99, mode)
    if not (mode == MASS and _ambiguous(margin, np.where(area > 0, wmax, 0))):
        assert float(tau_g.cpu()[0]) == tau_o
        assert (crit_g.cpu().numpy() == crit_o).all()


def test_pipeline_visibility_from_render(gpu_lib):
    """Per-view accumulations of a real render feed the visibility mask:
    every visible Gaussian contributes, and the mask culls in projection."""
    from tests.gpu_helpers import run_gpu_forward
    wl = gs_inputs.small_cube(seed=3)
    cams = wl.cameras
    res = run_gpu_forward(wl.scene, cams, per_view=True)
    imp = res["acc"]["importance"].view(len(cams), -1)
    vis, tau = D().visibility(imp)
    assert bool(((vis > 0) <= (imp > 0)).all())
    frac = (vis.sum(1).double() / (imp > 0).sum(1).clamp(min=1).double()).cpu().numpy()
    assert (frac > 0.2).all() and (frac <= 1.0).all()


@pytest.mark.parametrize("seed,n,k,use_area", [(0, 1, 1, False), (1, 5000, 1200, False), (2, 5000, 1200, True),
                                               (3, 100_003, 30_000, True), (4, 4096, 0, False),
                                               (5, 4096, 10_000, True), (6, 3_000_000, 1_500_000, True)])
def test_sample_matches_oracle(gpu_lib, seed, n, k, use_area):
    imp = gs_inputs.importance_like(1, n, seed)[0]
    expo = gs_inputs.exponential_draws(n, seed + 50)
    area = gs_inputs.wmax_like(n, seed + 60)[0] if use_area else None
    sel_g, cnt = D().sample(torch.from_numpy(imp).cuda(), torch.from_numpy(expo).cuda(), k,
                            None if area is None else torch.from_numpy(area.view(np.int32)).cuda())
    sel_o = oracle.sample(imp, expo, k, area)
    assert int(cnt.cpu()[0]) == int(sel_o.sum())
    assert (sel_g.cpu().numpy() == sel_o).all()


def test_sample_ties_by_index(gpu_lib):
    n = 10_000
    imp = np.ones(n, np.float32)
    expo = np.full(n, 0.75, np.float32)
    expo[::7] = 0.5
    for k in (1, 1000, 1429, 1430, 5000, n):
        sel_g, cnt = D().sample(torch.from_numpy(imp).cuda(), torch.from_numpy(expo).cuda(), k)
        sel_o = oracle.sample(imp, expo, k)
        assert (sel_g.cpu().numpy() == sel_o).all(), k
        assert int(cnt.cpu()[0]) == min(k, n)


@pytest.mark.parametrize("require_hit", [True, False])
@pytest.mark.parametrize("rate", [0.0, 0.05, 1.0])
def test_depth_points_matches_oracle(gpu_lib, require_hit, rate):
    cams = [gs_inputs.look_at((1.0, -2.0, 5.0), (0.2, 0.1, 0.0), 333, 201),
            gs_inputs.look_at((-4.0, 1.0, 2.0), (0.0, 0.0, 0.0), 64, 48)]
    sizes = [c.width * c.height for c in cams]
    P = sum(sizes)
    depth, imax, hit = gs_inputs.depth_map_like(P, 7)
    target = gs_inputs.uniform_image(3, P, 8)
    u = gs_inputs.uniform_draws(P, 9)
    t = lambda a: torch.from_numpy(a).cuda()
    pts, col, cnt = D().depth_points(t(depth), t(imax), t(hit), t(target), t(u), cams, rate, require_hit)
    m = int(cnt.cpu()[0])
    ref_p, ref_c, base = [], [], 0
    for c, sz in zip(cams, sizes):
        sl = slice(base, base + sz)
        p_, c_ = oracle.depth_points(c, depth[sl], imax[sl], hit[sl], target[:, sl], u[sl], rate, require_hit)
        ref_p.append(p_)
        ref_c.append(c_)
        base += sz
    ref_p = np.concatenate(ref_p)
    ref_c = np.concatenate(ref_c)
    assert m == ref_p.shape[0]
    got_p = pts[:, :m].cpu().numpy().T.astype(np.float64)
    np.testing.assert_allclose(got_p, ref_p, rtol=2e-6, atol=2e-6)
    assert (col[:, :m].cpu().numpy().T == ref_c.astype(np.float32)).all()


def test_depth_points_capacity(gpu_lib):
    cams = [gs_inputs.look_at((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 128, 96)]
    P = 128 * 96
    depth, imax, hit = gs_inputs.depth_map_like(P, 17)
    target = gs_inputs.uniform_image(3, P, 18)
    u = gs_inputs.uniform_draws(P, 19)
    t = lambda a: torch.from_numpy(a).cuda()
    pts, col, cnt = D().depth_points(t(depth), t(imax), t(hit), t(target), t(u), cams, 1.0, True, capacity=100)
    ref_p, _ = oracle.depth_points(cams[0], depth, imax, hit, target, u, 1.0, True)
    assert int(cnt.cpu()[0]) == ref_p.shape[0] > 100
    np.testing.assert_allclose(pts.cpu().numpy().T.astype(np.float64), ref_p[:100], rtol=2e-6, atol=2e-6)
