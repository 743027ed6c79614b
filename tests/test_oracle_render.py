"""Pins for the oracle's compositing (Eq. 1), argmax depth (Eq. 2), mid-point
depth (Sec. 4.1) and per-Gaussian accumulations (importance, area, max weight).
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import gs_inputs
import oracle
from oracle import F, brute
from tests.oracle_scenes import identity_camera, random_small_scene, scene_from

OPTS = oracle.Opts()


def _fwd(sc, cam, opts=OPTS, **kw):
    return oracle.forward_view(oracle.Params.of(sc), cam, opts, **kw)


def test_single_gaussian_at_pixel_centre():
    # C = rgb * o * 1, T_final = 1 - o, i_max = 0, mid-point depth = centre depth.
    f, z0, W, H = 32.0, 4.0, 32, 32
    cam = identity_camera(W, H, f, z0)
    x = (10.5 - 16.0) * z0 / f
    y = (7.5 - 16.0) * z0 / f
    o = 0.63
    rgb = np.array([0.25, 0.5, 0.75])
    sc = scene_from([x, y, 0.0], [0.05] * 3, [1, 0, 0, 0], [o], dc_rgb=[rgb])
    out = _fwd(sc, cam)
    p = 7 * W + 10
    P = out["proj"][0]
    assert P[F["U"]] == pytest.approx(10.5, abs=1e-5) and P[F["V"]] == pytest.approx(7.5, abs=1e-5)
    # the float32 position lands within 1e-5 px of the centre, where G = 1 - O(1e-10)
    o32 = float(np.float32(o))
    assert out["color"][p] == pytest.approx(o32 * np.array([P[F["R"]], P[F["G"]], P[F["B"]]]), rel=1e-9)
    assert out["t_final"][p] == pytest.approx(1 - o32, rel=1e-9)
    assert out["imax"][p] == 0 and out["n_contrib"][p] == 1 and out["hit"][p] == 1
    assert out["depth"][p] == pytest.approx(P[F["Z"]], rel=1e-9)
    # any other pixel: alpha = o exp(-d^T S'^-1 d / 2) with the closed form of an
    # off-axis isotropic Gaussian, S' = (f s/z)^2 (I + t t^T / z^2) + lowpass I
    k2 = (float(np.float32(f)) * float(np.float32(0.05)) / z0) ** 2
    tx, ty = float(np.float32(x)), float(np.float32(y))
    S = k2 * (np.eye(2) + np.outer([tx, ty], [tx, ty]) / z0 ** 2) + OPTS.lowpass * np.eye(2)
    Si = np.linalg.inv(S)
    for (px, py) in [(11, 7), (12, 9), (8, 5)]:
        dv = np.array([px + 0.5 - P[F["U"]], py + 0.5 - P[F["V"]]])
        a = o32 * math.exp(-0.5 * dv @ Si @ dv)
        q = py * W + px
        if a >= OPTS.alpha_min:
            assert out["color"][q, 1] == pytest.approx(a * P[F["G"]], rel=1e-9)
        else:
            assert out["color"][q, 1] == 0


def test_two_gaussians_same_centre_closed_form():
    f, z0, W, H = 32.0, 4.0, 32, 32
    cam = identity_camera(W, H, f, z0)
    c1, c2 = np.array([0.9, 0.1, 0.2]), np.array([0.1, 0.8, 0.3])
    o1, o2 = 0.4, 0.7
    p = 16 * W + 16  # Gaussians at world (0,0,*) project to (16, 16): pixel 15/16 corner
    for near_first in (True, False):
        z1, z2 = (0.0, 1.0) if near_first else (1.0, 0.0)
        sc = scene_from([[0.5 * z0 / f, 0.5 * z0 / f, z1], [0.5 * (z0 + 1 - z1 + z1) / f, 0, z2]],
                        [[0.05] * 3] * 2, [[1, 0, 0, 0]] * 2, [o1, o2], dc_rgb=[c1, c2])
        # put both exactly on pixel (16, 16)'s ray
        for k, z in enumerate((z1, z2)):
            sc.means[0, k] = np.float32(0.5 * (z0 + z) / f)
            sc.means[1, k] = np.float32(0.5 * (z0 + z) / f)
        out = _fwd(sc, cam)
        a1, a2 = float(np.float32(o1)), float(np.float32(o2))
        P = out["proj"]
        G = [math.exp(-0.5 * (P[k, F["CA"]] * (16.5 - P[k, F["U"]]) ** 2 + 2 * P[k, F["CB"]] *
                              (16.5 - P[k, F["U"]]) * (16.5 - P[k, F["V"]]) + P[k, F["CC"]] * (16.5 - P[k, F["V"]]) ** 2))
             for k in range(2)]
        al = [a1 * G[0], a2 * G[1]]
        first, second = (0, 1) if near_first else (1, 0)
        col = [np.array([P[k, F["R"]], P[k, F["G"]], P[k, F["B"]]]) for k in range(2)]
        expect = al[first] * col[first] + (1 - al[first]) * al[second] * col[second]
        assert out["color"][p] == pytest.approx(expect, rel=1e-12)
        assert out["imax"][p] == (first if al[first] >= (1 - al[first]) * al[second] else second)


def test_stop_rule_closed_form():
    # six o=0.8 Gaussians on one pixel ray at increasing depth: T = 0.2^k, the
    # sixth would take T below 1e-4, so five are included and T_final = 0.2^5.
    f, z0, W, H = 32.0, 4.0, 32, 32
    cam = identity_camera(W, H, f, z0)
    n = 6
    zs = np.linspace(0.0, 2.5, n)
    cols = gs_inputs.rng(3).uniform(0.1, 0.9, size=(n, 3))
    means = [[0.5 * (z0 + z) / f, 0.5 * (z0 + z) / f, z] for z in zs]
    sc = scene_from(means, [[0.04] * 3] * n, [[1, 0, 0, 0]] * n, [0.8] * n, dc_rgb=cols)
    out = _fwd(sc, cam)
    p = 16 * W + 16
    P = out["proj"]
    al = []
    for k in range(n):
        dx, dy = 16.5 - P[k, F["U"]], 16.5 - P[k, F["V"]]
        al.append(float(np.float32(0.8)) * math.exp(-0.5 * (P[k, F["CA"]] * dx * dx + P[k, F["CC"]] * dy * dy)))
    T = 1.0
    C = np.zeros(3)
    for k in range(5):
        C += al[k] * T * P[k, [F["R"], F["G"], F["B"]]]
        T *= 1 - al[k]
    assert T * (1 - al[5]) < OPTS.t_min < T
    assert out["n_contrib"][p] == 5
    assert out["t_final"][p] == pytest.approx(T, rel=1e-12)
    assert out["color"][p] == pytest.approx(C, rel=1e-12)


def test_skip_threshold():
    # a pixel where alpha sits just below / above 1/255 is skipped / included.
    # On the optical axis an isotropic Gaussian stays isotropic on screen:
    # var = (f s / z)^2 + lowpass; pick s so that alpha at the pixel is factor/255.
    f, z0, W, H = 32.0, 4.0, 64, 32
    cam = identity_camera(W, H, f, z0)
    o32 = float(np.float32(0.5))
    px, py = 36, 16
    d2 = (px + 0.5 - 32.0) ** 2 + (py + 0.5 - 16.0) ** 2
    for factor, drawn in ((0.98, False), (1.02, True)):
        var = -d2 / (2 * math.log(factor * OPTS.alpha_min / o32))
        s = math.sqrt(var - OPTS.lowpass) * z0 / f
        sc = scene_from([0.0, 0.0, 0.0], [s] * 3, [1, 0, 0, 0], [0.5], dc_rgb=[[1, 1, 1]])
        out = _fwd(sc, cam)
        val = out["color"][py * W + px, 0]
        assert (val > 0) == drawn
        if drawn:
            assert val == pytest.approx(factor * OPTS.alpha_min, rel=1e-5)


def _small_random(seed, n=48, W=40, H=32, degree=3):
    sc = random_small_scene(seed, n=n, spread=0.8, scale_lo=0.02, scale_hi=0.2, degree=degree)
    cam = gs_inputs.look_at((0.3, -0.2, 3.5), (0, 0, 0), W, H, 55.0)
    return sc, cam


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_matches_vectorised_restatement(seed):
    sc, cam = _small_random(seed)
    out = _fwd(sc, cam)
    P = out["proj"]
    col, tf, best, w, o = brute.composite(P[:, F["U"]], P[:, F["V"]], P[:, [F["CA"], F["CB"], F["CC"]]],
                                          P[:, F["OPAC"]], P[:, [F["R"], F["G"], F["B"]]], out["order"],
                                          cam.width, cam.height, OPTS.alpha_max, OPTS.alpha_min, OPTS.t_min,
                                          OPTS.bg)
    assert np.abs(col - out["color"]).max() < 1e-12
    assert np.abs(tf - out["t_final"]).max() < 1e-12
    assert np.array_equal(best, out["imax"])
    # accumulations: importance and max weight per Gaussian, area per argmax
    imp = np.zeros(sc.n)
    np.add.at(imp, o, w.sum(axis=0))
    assert np.abs(imp - out["importance"]).max() < 1e-12
    wm = np.zeros(sc.n)
    np.maximum.at(wm, o, w.max(axis=0))
    assert np.abs(wm - out["wmax"]).max() < 1e-15
    area = np.bincount(best[best >= 0], minlength=sc.n)
    assert np.array_equal(area, out["area"])


@pytest.mark.parametrize("seed", [5, 6])
def test_invariants(seed):
    sc = gs_inputs.uniform_cube_scene(600, seed, log_scale_mu=-3.0)
    cam = gs_inputs.look_at((0.0, 0.0, 4.0), (0, 0, 0), 72, 56, 60.0)
    out = _fwd(sc, cam)
    assert out["t_final"].min() >= OPTS.t_min and out["t_final"].max() <= 1.0
    # partition of unity: sum_i w_i + T_final = 1 per pixel, so sum_i I_i = sum_px (1 - T)
    assert out["importance"].sum() == pytest.approx((1 - out["t_final"]).sum(), rel=1e-12)
    assert out["area"].sum() == (out["imax"] >= 0).sum()
    assert np.all(out["wmax"] <= np.minimum(out["importance"], OPTS.alpha_max) + 1e-15)
    # blended depth equals sum of w * z; centre depth equals z of the argmax
    o1 = oracle.Opts(depth_mode=1)
    d1 = _fwd(sc, cam, o1)["depth"]
    zi = out["proj"][out["imax"], F["Z"]]
    assert np.array_equal(d1[out["imax"] >= 0], zi[out["imax"] >= 0])


def test_constant_colour_with_matching_background():
    sc = gs_inputs.uniform_cube_scene(300, 4, log_scale_mu=-2.5)
    sc.sh[:] = 0
    c = np.array([0.3, 0.55, 0.8])
    sc.sh[0] = ((c - 0.5) / (0.5 / math.sqrt(math.pi)))[:, None]
    cam = gs_inputs.look_at((0.0, 0.0, 4.0), (0, 0, 0), 48, 40, 60.0)
    out = _fwd(sc, cam, oracle.Opts(bg=tuple(c)))
    col_f = out["proj"][out["proj"][:, F["VALID"]] == 1][:, [F["R"], F["G"], F["B"]]]
    cc = col_f[0]
    assert np.abs(col_f - cc).max() < 1e-12
    assert np.abs(out["color"] - cc).max() < 1e-6  # cc == c up to float32 of the SH coefficient


@pytest.mark.parametrize("seed", [7, 8])
def test_tiled_equals_untiled(seed):
    # With the opacity-aware extent, restricting each pixel to its tile's list
    # drops only pairs with alpha < 1/255, so the outputs are identical.
    sc = gs_inputs.uniform_cube_scene(400, seed, log_scale_mu=-2.8)
    cam = gs_inputs.look_at((0.4, 0.3, 4.0), (0, 0, 0), 90, 70, 60.0)
    p = oracle.Params.of(sc)
    out = _fwd(sc, cam)
    proj = out["proj"]
    tx, ty, base, total = oracle.view_layout([cam])
    keys, vals, ranges = oracle.bin(oracle.tile_rects(proj), oracle.zbits(proj), 1, sc.n, base, tx, total)
    tiled = oracle.render(p, cam, proj, out["order"], OPTS, tiles=(vals, ranges.reshape(-1)))
    for k in ("color", "depth", "imax", "t_final", "n_contrib", "hit", "importance", "wmax", "area"):
        assert np.array_equal(tiled[k], out[k]), k


def test_mid_depth_sphere_closed_form():
    # isotropic Gaussian: t* is the foot of the perpendicular from the centre to
    # the ray; the ray meets the 1-sigma sphere iff its distance is <= s.
    cam = gs_inputs.look_at((0.5, 0.2, 5.0), (0, 0, 0), 64, 64, 50.0)
    s = 0.3
    sc = scene_from([0.05, -0.02, 0.1], [s] * 3, [0.3, 0.1, 0.5, 0.2], [0.95], dc_rgb=[[0.5] * 3])
    out = _fwd(sc, cam)
    R = cam.R.astype(np.float64)
    c = -R.T @ cam.t.astype(np.float64)
    p = sc.means[:, 0].astype(np.float64)
    sf = float(sc.scales[0, 0])
    checked = 0
    for pix in range(64 * 64):
        if out["imax"][pix] != 0:
            continue
        px, py = pix % 64, pix // 64
        d = R.T @ np.array([(px + 0.5 - cam.cx) / cam.fx, (py + 0.5 - cam.cy) / cam.fy, 1.0])
        tf = (p - c) @ d / (d @ d)
        rho = np.linalg.norm(c + tf * d - p)
        assert out["depth"][pix] == pytest.approx(tf, rel=1e-12)
        if abs(rho - sf) > 1e-9:
            assert out["hit"][pix] == (rho <= sf)
        checked += 1
    assert checked > 50


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_mid_depth_is_density_maximum_along_ray(seed):
    # anisotropic Gaussian: the mid-point equals the argmax of the 3D density on
    # the ray (golden-section search), and hit <=> that maximum is >= exp(-1/2).
    g = gs_inputs.rng(seed)
    cam = gs_inputs.look_at(g.normal(size=3) * 0 + np.array([1.0, -0.5, 4.5]), (0, 0, 0), 48, 48, 50.0)
    s = np.exp(g.normal(-1.6, 0.6, size=3))
    q = g.normal(size=4)
    sc = scene_from(g.uniform(-0.2, 0.2, size=3), s, q, [0.97], dc_rgb=[[0.5] * 3])
    out = _fwd(sc, cam)
    R = cam.R.astype(np.float64)
    c = -R.T @ cam.t.astype(np.float64)
    p = sc.means[:, 0].astype(np.float64)
    qf = sc.quats[:, 0].astype(np.float64)
    Rq = Rotation.from_quat([qf[1], qf[2], qf[3], qf[0]]).as_matrix()
    Ainv = Rq @ np.diag(1.0 / sc.scales[:, 0].astype(np.float64) ** 2) @ Rq.T
    rng_pix = [i for i in range(48 * 48) if out["imax"][i] == 0][::7]
    assert len(rng_pix) > 5
    for pix in rng_pix:
        px, py = pix % 48, pix // 48
        d = R.T @ np.array([(px + 0.5 - cam.cx) / cam.fx, (py + 0.5 - cam.cy) / cam.fy, 1.0])

        def m(t):
            e = c + t * d - p
            return e @ Ainv @ e

        lo, hi = 0.0, 20.0
        gr = (math.sqrt(5) - 1) / 2
        for _ in range(200):
            a1 = hi - gr * (hi - lo)
            a2 = lo + gr * (hi - lo)
            if m(a1) < m(a2):
                hi = a2
            else:
                lo = a1
        tmax = 0.5 * (lo + hi)
        assert out["depth"][pix] == pytest.approx(tmax, abs=1e-7)
        if abs(m(tmax) - 1) > 1e-9:
            assert out["hit"][pix] == (m(tmax) <= 1)


def test_empty_scene_and_background():
    cam = identity_camera(20, 12, 20.0, 3.0)
    sc = gs_inputs.uniform_cube_scene(0, 0)
    out = _fwd(sc, cam, oracle.Opts(bg=(0.1, 0.2, 0.3)))
    assert np.allclose(out["color"], [0.1, 0.2, 0.3]) and np.all(out["imax"] == -1)
    assert np.all(out["t_final"] == 1) and np.all(out["depth"] == 0)


def test_pixel_list_matches_full_image():
    sc, cam = _small_random(9)
    full = _fwd(sc, cam)
    pix = np.array([[3, 4], [39, 31], [20, 10], [0, 0]], dtype=np.int32)
    part = oracle.render(oracle.Params.of(sc), cam, full["proj"], full["order"], OPTS, pixels=pix)
    idx = pix[:, 1] * cam.width + pix[:, 0]
    for k in ("color", "depth", "imax", "t_final"):
        assert np.array_equal(part[k], full[k][idx])
