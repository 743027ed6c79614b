"""GPU (HIP, gfx950) parity against the FP64 oracle, through the C ABI.

Bit-exact: rectangles, tile keys, sorted order, per-tile ranges, sort of
synthetic pairs.  Colour, depth, transmittance: <= 1e-4 max abs on every
pixel, against the definition or, where a decision of Eq. (1)-(2) sits within
float32 rounding of its threshold, against the branch the pixel took.
Accumulations under the same branches: area exact, importance and max weight
<= 1e-5 relative for every Gaussian.  Gradients: <= 1e-3 relative L2 per
parameter group, with the oracle following the same branches.
"""
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


def _oracle_view(scene, cam, opts=None, cull=None, pixels=None):
    p = oracle.Params.of(scene)
    return p, oracle.forward_view(p, cam, opts or oracle.Opts(), cull_mask=cull, pixels=pixels)


def _small(seed=0, n=4096, W=128, H=128):
    return gs_inputs.small_cube(seed, n, W, H)


# ---------------------------------------------------------------------------
def test_project_matches_oracle(gpu_lib):
    wl = _small()
    out = H.run_gpu_forward(wl.scene, wl.cameras, accumulate=False)
    rec, binr = _np(out["proj"].rec).astype(np.float64), _np(out["proj"].bin)
    _, orc = _oracle_view(wl.scene, wl.cameras[0])
    P = orc["proj"]
    vis_o = (P[:, F["VALID"]] == 1) & (P[:, F["TILES"]] > 0)
    vis_g = binr[:, 3] > 0
    assert np.array_equal(vis_o, vis_g)
    v = vis_o
    u = rec[:, 0] + rec[:, 2]
    vv = rec[:, 1] + rec[:, 3]
    assert np.abs(u[v] - P[v, F["U"]]).max() < 1e-6 and np.abs(vv[v] - P[v, F["V"]]).max() < 1e-6
    for k, f in ((13, "CA"), (14, "CB"), (15, "CC")):
        scale = np.abs(P[v, F["CA"]]) + np.abs(P[v, F["CC"]])
        assert (np.abs(rec[v, k] - P[v, F[f]]) / scale).max() < 1e-6
    for k, f in ((8, "R"), (9, "G"), (10, "B")):
        assert np.abs(rec[v, k] - P[v, F[f]]).max() < 1e-6
    assert np.array_equal(rec[v, 12].astype(np.float32), P[v, F["Z"]].astype(np.float32))
    box = np.stack([binr[:, 0] & 0xFFFF, binr[:, 0] >> 16, binr[:, 1] & 0xFFFF, binr[:, 1] >> 16], 1)
    obox = P[:, [F["XLO"], F["XHI"], F["YLO"], F["YHI"]]].astype(np.int64)
    assert np.array_equal(box[v], obox[v])
    assert np.array_equal(binr[v, 3], P[v, F["TILES"]].astype(np.int64))
    assert np.array_equal(binr[v, 2].view(np.uint32), P[v, F["Z"]].astype(np.float32).view(np.uint32))


@pytest.fixture(params=["fold", "top scan"])
def count_path(request):
    """gs_bin_count's two paths: the down-sweep adding the earlier blocks'
    totals itself (the default at these sizes), or a scan kernel between."""
    from paper_2411_12788_amd import _lib as L
    lib = L.lib()
    prev = lib.gs_bin_count_set_fold_blocks(0 if request.param == "top scan" else -1)
    yield request.param
    lib.gs_bin_count_set_fold_blocks(prev)


def test_binning_bit_exact(gpu_lib, count_path):
    wl = _small(seed=1)
    out = H.run_gpu_forward(wl.scene, wl.cameras, accumulate=False, want_keys=True)
    b = out["binned"]
    _, orc = _oracle_view(wl.scene, wl.cameras[0])
    P = orc["proj"]
    tx, ty, base, total = oracle.view_layout(wl.cameras)
    keys, vals, ranges = oracle.bin(oracle.tile_rects(P), oracle.zbits(P), 1, wl.scene.n, base, tx, total)
    assert b.stats.n_isect == len(keys)
    assert np.array_equal(_np(b.keys).view(np.uint64), keys)
    assert np.array_equal(_np(b.vals).view(np.uint32), vals)
    assert np.array_equal(_np(b.ranges).view(np.uint32), ranges)
    H.check_bin_extras(b, oracle.tile_rects(P), oracle.zbits(P), 1, total, ranges, "small")


@pytest.mark.parametrize("which", ["cube 4096 128x128", "surfaces 500k 1245x825"])
def test_split_binning_stages_match_oracle(gpu_lib, which, count_path):
    """gs_emit_keys, gs_sort_pairs and gs_tile_ranges called one by one give
    the oracle's sorted keys (as (tile << 32) | z bits), values and ranges;
    keys_out may not be the keys themselves."""
    import ctypes
    from paper_2411_12788_amd import _lib as L
    R = H.raster()
    lib = L.lib()
    wl = _small(seed=3) if which.startswith("cube") else gs_inputs.training_view()
    cams = wl.cameras
    ds = R.DeviceScene.from_numpy(wl.scene)
    n = ds.n
    proj = R.project(ds, cams, R.RasterOpts())
    offsets, st = R.bin_count(proj, cams, n)
    ni, tiles = int(st.n_isect), int(st.tiles_total)
    print("split binning case:", which, count_path, ni, "pairs", flush=True)
    keys = torch.empty(ni, dtype=torch.int64, device="cuda")
    vals = torch.empty(ni, dtype=torch.int32, device="cuda")
    assert lib.gs_emit_keys(ctypes.byref(proj.c()), R.cameras(cams), len(cams), n, R._ptr(offsets), st.depth_bits,
                            st.zbits_min, R._ptr(keys), R._ptr(vals), None) == L.GS_OK
    ws = torch.empty(lib.gs_sort_workspace_size(ni), dtype=torch.uint8, device="cuda")
    assert lib.gs_sort_pairs(R._ptr(keys), R._ptr(vals), ni, st.key_bits, R._ptr(ws), ws.numel(), None) == L.GS_OK
    ranges = torch.full((tiles, 2), 7, dtype=torch.int32, device="cuda")
    kout = torch.empty(ni, dtype=torch.int64, device="cuda")
    assert lib.gs_tile_ranges(R._ptr(keys), ni, st.depth_bits, st.zbits_min, tiles, R._ptr(ranges), R._ptr(kout),
                              None) == L.GS_OK
    assert lib.gs_tile_ranges(R._ptr(keys), ni, st.depth_bits, st.zbits_min, tiles, R._ptr(ranges), R._ptr(keys),
                              None) == L.GS_ERR_SHAPE
    torch.cuda.synchronize()
    P = oracle.project(oracle.Params.of(wl.scene), cams[0], oracle.Opts())
    tx, ty, base, total = oracle.view_layout(cams)
    okeys, ovals, oranges = oracle.bin(oracle.tile_rects(P), oracle.zbits(P), 1, n, base, tx, total)
    assert ni == len(okeys) and tiles == total
    assert np.array_equal(_np(kout).view(np.uint64), okeys)
    assert np.array_equal(_np(vals).view(np.uint32), ovals)
    assert np.array_equal(_np(ranges).view(np.uint32), oranges)
    b = R.Binned(vals, ranges, kout, st, offsets, None)
    H.check_bin_extras(b, oracle.tile_rects(P), oracle.zbits(P), 1, total, oranges, which)


@pytest.mark.parametrize("algorithm", [0, 1])  # GS_SORT_PRESCAN, GS_SORT_LOOKBACK
@pytest.mark.parametrize("n,bits,spread", [(1, 8, 2), (1000, 20, 16), (3 * 4096 + 17, 45, 1 << 40),
                                           (100_003, 64, 1 << 62), (50_000, 33, 7), (3_300_001, 45, 1 << 44)])
def test_sort_pairs_matches_lexsort(gpu_lib, n, bits, spread, algorithm):
    from paper_2411_12788_amd import _lib as L
    R = H.raster()
    g = gs_inputs.rng(n + bits)
    hi = min(spread, (1 << bits) - 1) if bits < 64 else spread
    keys = g.integers(0, hi, size=n, dtype=np.uint64, endpoint=True)
    if bits < 64:
        keys &= np.uint64((1 << bits) - 1)
    vals = np.arange(n, dtype=np.uint32)
    kt = torch.from_numpy(keys.view(np.int64)).cuda()
    vt = torch.from_numpy(vals.view(np.int32)).cuda()
    assert L.lib().gs_sort_set_algorithm(algorithm) == L.GS_OK
    try:
        R.sort_pairs(kt, vt, bits)
        torch.cuda.synchronize()
    finally:
        L.lib().gs_sort_set_algorithm(L.GS_SORT_PRESCAN)
    perm = np.lexsort((vals, keys))
    assert np.array_equal(_np(kt).view(np.uint64), keys[perm])
    assert np.array_equal(_np(vt).view(np.uint32), vals[perm])


def test_forward_and_accumulations_small_cube(gpu_lib):
    wl = _small(seed=2)
    cam = wl.cameras[0]
    out = H.run_gpu_forward(wl.scene, wl.cameras, accumulate=True)
    p, orc = _oracle_view(wl.scene, cam)
    flips, _ = H.compare_forward(out["frame"], orc, slice(0, 128 * 128), "small cube", p, cam)
    H.check_accum(out["acc"], p, cam, orc["proj"], orc["order"], oracle.Opts(), flips, wl.scene.n, "small cube")
    # invariants on the GPU's own outputs
    imp = _np(out["acc"]["importance"]).astype(np.float64)
    tf = _np(out["frame"].t_final).astype(np.float64)
    assert imp.sum() == pytest.approx((1 - tf).sum(), rel=1e-5)
    assert int(_np(out["acc"]["area"]).sum()) == int((_np(out["frame"].imax) >= 0).sum())


def test_accumulate_importance_equals_fused(gpu_lib):
    R = H.raster()
    wl = _small(seed=3)
    out = H.run_gpu_forward(wl.scene, wl.cameras, accumulate=True)
    acc2 = R.alloc_accum(wl.scene.n)
    R.accumulate_importance(out["proj"], out["binned"], wl.cameras, wl.scene.n, R.RasterOpts(), acc2)
    torch.cuda.synchronize()
    assert np.array_equal(_np(acc2["area"]), _np(out["acc"]["area"]))
    assert np.array_equal(_np(acc2["wmax"]), _np(out["acc"]["wmax"]))
    assert np.allclose(_np(acc2["importance"]), _np(out["acc"]["importance"]), rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("depth_mode", [1, 2])
def test_depth_modes(gpu_lib, depth_mode):
    R = H.raster()
    wl = _small(seed=4, n=2048, W=96, H=80)
    out = H.run_gpu_forward(wl.scene, wl.cameras, opts=R.RasterOpts(depth_mode=depth_mode), accumulate=False)
    o = oracle.Opts(depth_mode=depth_mode)
    p, orc = _oracle_view(wl.scene, wl.cameras[0], o)
    H.compare_forward(out["frame"], orc, slice(0, 96 * 80), f"depth mode {depth_mode}", p, wl.cameras[0], o)


def _grads_np(g, n):
    return {k: _np(v)[..., :n].astype(np.float64) for k, v in g.items()}


@pytest.mark.parametrize("masked", [False, True])
def test_backward_small_cube(gpu_lib, masked):
    R = H.raster()
    wl = _small(seed=5, n=3000, W=112, H=96)
    cam = wl.cameras[0]
    out = H.run_gpu_forward(wl.scene, wl.cameras, accumulate=False)
    p, orc = _oracle_view(wl.scene, cam)
    flips, _ = H.compare_forward(out["frame"], orc, slice(0, cam.width * cam.height), "backward cube", p, cam)
    Pn = cam.width * cam.height
    dldc = gs_inputs.normal_image(3, Pn, 77, scale=1.0 / Pn)
    active = gs_inputs.bernoulli_mask(wl.scene.n, 0.25, 78) if masked else None
    grads, g2d = R.render_backward(out["scene"], out["proj"], out["binned"], wl.cameras, R.RasterOpts(),
                                   out["frame"], torch.from_numpy(dldc).cuda(),
                                   None if active is None else torch.from_numpy(active).cuda())
    torch.cuda.synchronize()
    og, og2d = H.backward_views(p, wl.cameras, oracle.Opts(), [dldc.T.astype(np.float64)], active=active,
                                flips=[flips])
    gg = _grads_np(grads, wl.scene.n)
    for k in ("means", "scales", "quats", "opacity", "sh"):
        err = H.rel_l2(gg[k], og[k])
        assert err <= H.GRAD_REL_L2, (k, err)
        if masked:
            assert np.all(gg[k][..., active == 0] == 0), k
    g2 = _np(g2d).astype(np.float64)[: wl.scene.n]
    ref = og2d[0] if not masked else og2d[0] * active[:, None]
    assert H.rel_l2(g2, ref) <= H.GRAD_REL_L2
    if masked:
        assert np.all(g2[active == 0] == 0)


@pytest.mark.parametrize("case", ["needles", "cube masked", "needles two views"])
def test_projection_backward_alone(gpu_lib, case):
    """a8 by itself: parameters from the GPU's own per-record 2D gradient,
    against the oracle's chain rule of that same gradient.  Needle-like
    Gaussians (one axis 12x the others) are where an unfortunate order of the
    float chain rule loses most (forming the 2D covariance gradient first
    cancels by the elongation squared); two views take the multi-view kernel."""
    R = H.raster()
    if case == "cube masked":
        wl = _small(seed=25, n=3000, W=112, H=96)
        cams = wl.cameras
        active = gs_inputs.bernoulli_mask(wl.scene.n, 0.25, 26)
    else:
        wl = gs_inputs.elongated_cube(seed=27)
        cams = wl.cameras if case == "needles" else [wl.cameras[0], gs_inputs.look_at((1.5, 0.5, 3.5), (0, 0, 0),
                                                                                       144, 112)]
        active = None
    lay = R.view_layout(cams)
    out = H.run_gpu_forward(wl.scene, cams, accumulate=False)
    dldc = torch.from_numpy(gs_inputs.normal_image(3, lay.pixels_total, 28, scale=1.0 / lay.pixels_total)).cuda()
    grads, g2d = R.render_backward(out["scene"], out["proj"], out["binned"], cams, R.RasterOpts(), out["frame"],
                                   dldc, None if active is None else torch.from_numpy(active).cuda())
    torch.cuda.synchronize()
    H.check_projection_backward(oracle.Params.of(wl.scene), cams, oracle.Opts(), _np(g2d),
                                _grads_np(grads, wl.scene.n), wl.scene.n, active=active, what=case)


def test_multiview_mixed_resolution(gpu_lib):
    R = H.raster()
    sc = gs_inputs.uniform_cube_scene(2500, 9)
    cams = [gs_inputs.look_at((0, 0, 4), (0, 0, 0), 96, 64), gs_inputs.look_at((2.5, 1, 3), (0, 0, 0), 50, 37),
            gs_inputs.look_at((-3, 0.5, 2.5), (0, 0, 0), 128, 80)]
    out = H.run_gpu_forward(sc, cams, accumulate=True, per_view=True)
    lay = R.view_layout(cams)
    p = oracle.Params.of(sc)
    dls, fls = [], []
    n = sc.n
    for v, cam in enumerate(cams):
        orc = oracle.forward_view(p, cam, oracle.Opts())
        sl = slice(lay.pixel_base[v], lay.pixel_base[v] + cam.width * cam.height)
        flips, _ = H.compare_forward(out["frame"], orc, sl, f"view {v}", p, cam)
        accv = {k: t[v * n:(v + 1) * n] for k, t in out["acc"].items()}
        H.check_accum(accv, p, cam, orc["proj"], orc["order"], oracle.Opts(), flips, n, f"view {v}")
        fls.append(flips)
        dls.append(gs_inputs.normal_image(3, cam.width * cam.height, 100 + v, scale=1e-3))
    dl = torch.from_numpy(np.concatenate(dls, axis=1)).cuda()
    grads, _ = R.render_backward(out["scene"], out["proj"], out["binned"], cams, R.RasterOpts(), out["frame"], dl)
    torch.cuda.synchronize()
    og, _ = H.backward_views(p, cams, oracle.Opts(), [d.T.astype(np.float64) for d in dls], flips=fls)
    gg = _grads_np(grads, n)
    for k in og:
        assert H.rel_l2(gg[k], og[k]) <= H.GRAD_REL_L2, k


def test_edge_cases(gpu_lib):
    R = H.raster()
    cam = gs_inputs.look_at((0, 0, 4), (0, 0, 0), 37, 23)
    # empty scene: background everywhere
    empty = gs_inputs.uniform_cube_scene(0, 0)
    opts = R.RasterOpts(bg=(0.25, 0.5, 0.75))
    out = H.run_gpu_forward(empty, [cam], opts=opts)
    assert np.allclose(_np(out["frame"].color).T, [0.25, 0.5, 0.75]) and np.all(_np(out["frame"].imax) == -1)
    # all culled by the mask
    sc = gs_inputs.uniform_cube_scene(500, 3)
    out = H.run_gpu_forward(sc, [cam], opts=opts, cull=np.zeros(500, np.uint8))
    assert out["binned"].stats.n_isect == 0 and np.all(_np(out["frame"].t_final) == 1)
    # partial cull mask and lower SH degrees against the oracle
    cull = gs_inputs.bernoulli_mask(500, 0.6, 4)
    for deg in (0, 1, 2):
        sc.sh_degree = deg
        out = H.run_gpu_forward(sc, [cam], opts=opts, cull=cull)
        o = oracle.Opts(bg=(0.25, 0.5, 0.75))
        p, orc = _oracle_view(sc, cam, o, cull=cull)
        H.compare_forward(out["frame"], orc, slice(0, 37 * 23), f"deg {deg}", p, cam, o)
    sc.sh_degree = 3


def test_argument_errors(gpu_lib):
    import ctypes
    from paper_2411_12788_amd import _lib as L
    lib = L.lib()
    R = H.raster()
    cams = R.cameras([gs_inputs.look_at((0, 0, 4), (0, 0, 0), 16, 16)])
    o = R.RasterOpts().c()
    outp = L.Projected()
    assert lib.gs_project(None, cams, 1, None, ctypes.byref(o), ctypes.byref(outp), None) == L.GS_ERR_NULL
    ds = R.DeviceScene.from_numpy(gs_inputs.uniform_cube_scene(8, 0))
    assert lib.gs_project(ctypes.byref(ds.c()), cams, 0, None, ctypes.byref(o), ctypes.byref(outp), None) == \
        L.GS_ERR_SHAPE
    cams[0].fx = float("nan")
    assert lib.gs_project(ctypes.byref(ds.c()), cams, 1, None, ctypes.byref(o), ctypes.byref(outp), None) == \
        L.GS_ERR_CAMERA


def test_l1_loss_grad_matches_definition(gpu_lib):
    R = H.raster()
    # up to a 1080p frame and many passes of the capped grid (256 x 1024
    # threads, one float4 each per pass); `skew` offsets the buffers by one
    # float, off the 16-byte alignment of the float4 path
    for count, skew in ((1, 0), (7, 0), (4099, 0), (3 * 128 * 96 + 2, 0), (3 * 1920 * 1080, 0),
                        (4 * 4096 * 256 * 4 + 4 * 999 + 3, 0), (3 * 1920 * 1080 - 5, 1)):
        g = gs_inputs.rng(count)
        c = torch.from_numpy(g.uniform(size=count + skew).astype(np.float32)).cuda()[skew:]
        t = torch.from_numpy(g.uniform(size=count + skew).astype(np.float32)).cuda()[skew:]
        t[: count // 5] = c[: count // 5]  # exact ties give a zero gradient
        dl = torch.empty(count + skew, device="cuda")[skew:]
        loss = torch.zeros(1, device="cuda")
        R.l1_loss_grad(c, t, dl, loss)
        torch.cuda.synchronize()
        d = (c - t).double().cpu().numpy()
        assert np.array_equal(_np(dl), (np.sign(d) / count).astype(np.float32))
        assert loss.item() == pytest.approx(np.abs(d).mean(), rel=1e-5)


def test_fill_u32_writes_exactly_its_words(gpu_lib):
    """16-byte stores over the aligned part, word stores elsewhere: every word
    of the range takes the value, the words around it keep theirs."""
    R = H.raster()
    for count, skew in ((1, 0), (3, 1), (4, 0), (5, 3), (4099, 2), (8192 * 256 * 4 * 3 + 7, 1),
                        (36 * 10 ** 6 + 1, 0)):
        buf = torch.full((count + skew + 4,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
        R.fill_u32(buf[skew: skew + count], 0xC0FFEE)
        torch.cuda.synchronize()
        b = _np(buf).view(np.uint32)
        assert np.all(b[skew: skew + count] == 0xC0FFEE), (count, skew)
        assert np.all(b[:skew] == 0x5A5A5A5A) and np.all(b[skew + count:] == 0x5A5A5A5A), (count, skew)


def test_tile_order_is_longest_first_permutation(gpu_lib):
    wl = _small(seed=6)
    out = H.run_gpu_forward(wl.scene, wl.cameras, accumulate=False)
    b = out["binned"]
    order = _np(b.order).astype(np.int64)
    rng = _np(b.ranges).view(np.uint32).astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(len(rng)))
    lengths = rng[order, 1] - rng[order, 0]
    bits = np.where(lengths > 0, np.floor(np.log2(np.maximum(lengths, 1))) + 1, 0)
    assert np.all(np.diff(bits) <= 0)


def test_fused_binning_equals_two_calls(gpu_lib):
    """gs_bin through raster.bin_step: the first call (empty buffers: the
    sort runs as a second call after they grow), a repeat (everything in one
    call), a larger workload (growth again) and a smaller one (one call into
    larger buffers) give the lists of the separate count and sort; an empty
    scene gives empty ranges."""
    R = H.raster()
    bufs = R.StepBuffers()
    for seed, n in ((21, 4096), (21, 4096), (22, 9000), (23, 1000), (24, 0)):
        wl = _small(seed=seed, n=max(n, 1))
        if n == 0:
            wl.scene.opacity[:] = 0.0  # nothing reaches alpha_min: no pairs
        opts = R.RasterOpts()
        ds = R.DeviceScene.from_numpy(wl.scene)
        proj = R.project(ds, wl.cameras, opts)
        fused = R.bin_step(proj, wl.cameras, ds.n, bufs, want_keys=True)
        fresh = R.bin(proj, wl.cameras, ds.n, want_keys=True)
        torch.cuda.synchronize()
        assert fused.stats.n_isect == fresh.stats.n_isect
        assert torch.equal(fused.keys, fresh.keys)
        assert torch.equal(fused.vals, fresh.vals)
        assert torch.equal(fused.ranges, fresh.ranges)
        assert torch.equal(fused.order, fresh.order)
        assert torch.equal(fused.offsets, fresh.offsets)
        if n == 0:
            assert fused.stats.n_isect == 0 and int(fused.ranges.abs().sum()) == 0


def test_bin_buffers_reused_across_sizes(gpu_lib):
    """Binning into reused buffers (larger, then smaller, then larger again)
    gives the same lists as fresh buffers."""
    R = H.raster()
    bufs = R.BinBuffers()
    for seed, n in ((11, 4096), (12, 1000), (13, 6000)):
        wl = _small(seed=seed, n=n)
        opts = R.RasterOpts()
        ds = R.DeviceScene.from_numpy(wl.scene)
        proj = R.project(ds, wl.cameras, opts)
        offsets, st = R.bin_count(proj, wl.cameras, n)
        reused = R.bin_sort(proj, wl.cameras, n, offsets, st, buffers=bufs)
        fresh = R.bin_sort(proj, wl.cameras, n, offsets, st)
        torch.cuda.synchronize()
        assert torch.equal(reused.vals, fresh.vals)
        assert torch.equal(reused.ranges, fresh.ranges)
        # the order inside a bit-length group is unspecified: compare the groups
        L = (fresh.ranges[:, 1] - fresh.ranges[:, 0]).long().cpu()
        bl = lambda o: [int(x).bit_length() for x in L[o.long().cpu()]]
        assert bl(reused.order) == bl(fresh.order)
        assert torch.equal(torch.sort(reused.order).values, torch.sort(fresh.order).values)

