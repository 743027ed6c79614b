"""GPU parity of the spatial order (the Morton layout the library stores
Gaussians in) and of the planar permutation, against the oracle; and the
property that makes the layout free: rendering and differentiating the
permuted scene gives the same results, moved by the permutation."""
import numpy as np
import pytest
import torch

import gs_inputs
import oracle
from tests.gpu_helpers import raster

pytestmark = pytest.mark.gpu
FULL = (1 << 30) - 1


def _gpu_order(means):
    R = raster()
    m = torch.from_numpy(np.ascontiguousarray(means, dtype=np.float32)).cuda()
    perm, codes = R.spatial_order(m, codes=True)
    torch.cuda.synchronize()
    return codes.cpu().numpy().view(np.uint32), perm.cpu().numpy().astype(np.int64)


def _check(means, what):
    print("spatial order case:", what, means.shape, flush=True)
    c_g, p_g = _gpu_order(means)
    c_o, p_o = oracle.spatial_order(means)
    bad = np.flatnonzero(c_g != c_o)
    assert bad.size == 0, (what, bad[:8].tolist(), c_g[bad[:4]].tolist(), c_o[bad[:4]].tolist())
    assert np.array_equal(p_g, p_o), (what, int((p_g != p_o).sum()))


def _special(kind):
    g = gs_inputs.rng(21)
    if kind == "nonfinite":
        m = g.uniform(-2, 2, size=(3, 5000)).astype(np.float32)
        rows = g.choice(5000, 40, replace=False)
        m[g.integers(0, 3, 40), rows] = np.array([np.nan, np.inf, -np.inf], np.float32)[g.integers(0, 3, 40)]
        return m
    if kind == "equal":
        return np.full((3, 3000), -1.25, np.float32)
    if kind == "big_extent":
        m = g.uniform(-1, 1, size=(3, 1000)).astype(np.float32)
        m[0, 0], m[0, 1] = -3e38, 3e38
        return m
    if kind == "grid_ties":
        return g.integers(-3, 3, size=(3, 70_000)).astype(np.float32)  # many equal codes
    if kind == "all_nonfinite":
        return np.full((3, 300), np.nan, np.float32)
    raise ValueError(kind)


@pytest.mark.parametrize("n", [1, 2, 255, 256, 257, 4097, 65_537])
def test_spatial_order_ragged_sizes(gpu_lib, n):
    _check(gs_inputs.uniform_cube_scene(n, 30 + n).means, f"cube n={n}")


@pytest.mark.parametrize("kind", ["nonfinite", "equal", "big_extent", "grid_ties", "all_nonfinite"])
def test_spatial_order_special_cases(gpu_lib, kind):
    _check(_special(kind), kind)


def test_spatial_order_surface_scenes(gpu_lib):
    _check(gs_inputs.training_view().scene.means, "surfaces 500k")
    _check(gs_inputs.large_scene().scene.means, "surfaces 3M")


def test_spatial_order_empty(gpu_lib):
    R = raster()
    perm = R.spatial_order(torch.empty((3, 0), device="cuda"))
    torch.cuda.synchronize()
    assert perm.numel() == 0


@pytest.mark.parametrize("dtype,shape", [(torch.uint8, (5000,)), (torch.float16, (2, 4099)),
                                         (torch.float32, (48, 3001)), (torch.float32, (3, 1)),
                                         (torch.int64, (3, 777))])
def test_permute_matches_indexing(gpu_lib, dtype, shape):
    R = raster()
    g = gs_inputs.rng(40)
    n = shape[-1]
    src = torch.from_numpy(g.integers(0, 100, size=shape).astype(np.int64)).to(dtype).cuda()
    perm_np = g.permutation(n).astype(np.int64)
    bad = g.choice(n, min(n, 5), replace=False)
    perm_np[bad[: len(bad) // 2]] = n + 3       # beyond n
    perm_np[bad[len(bad) // 2:]] = -1           # 2^32 - 1 as the library's u32
    perm = torch.from_numpy(perm_np.astype(np.int32)).cuda()
    out = R.permute(src, perm).cpu()
    ok = (perm_np >= 0) & (perm_np < n)
    ref = torch.zeros_like(src.cpu())
    ref[..., torch.from_numpy(np.flatnonzero(ok))] = src.cpu()[..., torch.from_numpy(perm_np[ok])]
    assert torch.equal(out, ref)


def _pipeline(ds, cams, active, dldc):
    R = raster()
    opts = R.RasterOpts()
    proj = R.project(ds, cams, opts)
    binned = R.bin(proj, cams, ds.n, want_keys=True)
    acc = R.alloc_accum(ds.n)
    frame = R.render_forward(ds, proj, binned, cams, opts, accum=acc)
    grads, _ = R.render_backward(ds, proj, binned, cams, opts, frame, dldc, active, deterministic=True)
    torch.cuda.synchronize()
    return binned, frame, acc, grads


@pytest.mark.parametrize("which", ["cube 4096 128x128", "surfaces 60k 320x240"])
def test_results_follow_the_permutation(gpu_lib, which):
    R = raster()
    if which.startswith("cube"):
        wl = gs_inputs.small_cube()
        scene, cams = wl.scene, wl.cameras
    else:
        scene = gs_inputs.surface_scene(60_000, 41)
        cams = gs_inputs.sphere_cameras(1, 6.0, [(320, 240)], 42)
        # keep one Gaussian per float32 camera depth, so that no two entries of
        # a list tie (tied entries keep index order and may change places)
        c = cams[0]
        z = (c.R.astype(np.float64) @ scene.means.astype(np.float64) + c.t.astype(np.float64)[:, None])[2]
        _, first = np.unique(z.astype(np.float32), return_index=True)
        scene = scene.subset(np.sort(first))
    n = scene.n
    print("permutation invariance case:", which, flush=True)
    ds = R.DeviceScene.from_numpy(scene)
    perm = R.spatial_order(ds.means)
    ds2 = ds.permuted(perm)
    active = torch.from_numpy(gs_inputs.bernoulli_mask(n, 0.5, 43)).cuda()
    active2 = R.permute(active, perm)
    P = R.view_layout(cams).pixels_total
    dldc = torch.from_numpy(gs_inputs.normal_image(3, P, 44)).cuda()
    b1, f1, a1, g1 = _pipeline(ds, cams, active, dldc)
    _, f2, a2, g2 = _pipeline(ds2, cams, active2, dldc)
    pl = perm.long()
    # entries of equal depth in one tile's list could change places: the case
    # must have none (no two equal consecutive sorted keys)
    k = b1.keys.cpu()
    assert k.numel() > 1000 and bool((k[1:] != k[:-1]).all()), "equal (tile, depth) keys"
    assert torch.equal(f1.color, f2.color)
    assert torch.equal(f1.t_final, f2.t_final)
    assert torch.equal(f1.depth, f2.depth)
    hit = f2.imax >= 0
    assert torch.equal(f1.imax >= 0, hit)
    assert torch.equal(f1.imax[hit].long(), pl[f2.imax[hit].long()])
    assert torch.equal(a1["area"][pl], a2["area"])
    assert torch.equal(a1["wmax"][pl], a2["wmax"])
    torch.testing.assert_close(a1["importance"][pl], a2["importance"], rtol=1e-6, atol=1e-7)
    for k in g1:
        assert torch.equal(g1[k][..., pl], g2[k]), k


def test_densify_reorder_moves_rows_with_the_scene(gpu_lib):
    """densify.reorder: the scene and per-Gaussian arrays of any shape and
    element size move by the same permutation, the spatial order of the means."""
    R = raster()
    from paper_2411_12788_amd import densify as D
    sc = gs_inputs.surface_scene(50_000, 45)
    ds = R.DeviceScene.from_numpy(sc)
    n = ds.n
    g = torch.Generator(device="cuda").manual_seed(46)
    adam = torch.randn((2, 59, n), device="cuda", generator=g)      # optimizer moments, planar
    count = torch.randint(0, 100, (n,), device="cuda", dtype=torch.int32, generator=g)
    flags = torch.randint(0, 2, (n,), device="cuda", dtype=torch.uint8, generator=g)
    out, (a2, c2, f2), perm = D.reorder(ds, adam, count, flags)
    torch.cuda.synchronize()
    assert torch.equal(perm, R.spatial_order(ds.means))
    p = perm.long()
    assert torch.equal(out.means, ds.means[:, p]) and torch.equal(out.scales, ds.scales[:, p])
    assert torch.equal(out.quats, ds.quats[:, p]) and torch.equal(out.opacity, ds.opacity[p])
    assert torch.equal(out.sh, ds.sh[..., p]) and out.sh_degree == ds.sh_degree
    assert torch.equal(a2, adam[..., p]) and torch.equal(c2, count[p]) and torch.equal(f2, flags[p])
