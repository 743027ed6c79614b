"""Pins for the oracle's analytic gradients: central finite differences of the
oracle's own forward in FP64 (a different computation: perturb, re-render,
difference), plus closed forms for a single Gaussian.
"""
import math

import numpy as np
import pytest

import gs_inputs
import oracle
from oracle import F
from tests.oracle_scenes import identity_camera, random_small_scene, scene_from

OPTS = oracle.Opts()


def _loss(params, cam, dldc, opts=OPTS, cull=None):
    out = oracle.forward_view(params, cam, opts, cull_mask=cull, accumulate=False)
    return float((out["color"] * dldc).sum()), out


def _margins_ok(params, cam, out, opts=OPTS):
    P = out["proj"]
    v = P[:, F["VALID"]] == 1
    z = np.sort(P[v, F["Z"]])
    zgap = np.diff(z).min() / z.max() if len(z) > 1 else 1.0
    raw = np.abs(P[v][:, [F["RAW_R"], F["RAW_G"], F["RAW_B"]]]).min()
    limx = opts.jac_clamp * cam.width / (2 * cam.fx)
    limy = opts.jac_clamp * cam.height / (2 * cam.fy)
    jm = min(np.abs(np.abs(P[v, F["TXTZ"]]) - limx).min(), np.abs(np.abs(P[v, F["TYTZ"]]) - limy).min())
    m = out["margin"]
    return dict(decision=min(m[:, 0].min(), m[:, 1].min()), clamp=m[:, 3].min(), zgap=zgap, raw=raw, jac=jm)


def _fd(params, cam, dldc, name, idx, h_rel=1e-6, cull=None):
    arr = getattr(params, name)
    x0 = arr[idx]
    h = h_rel * max(1.0, abs(x0))
    p1 = params.copy()
    getattr(p1, name)[idx] = x0 + h
    p2 = params.copy()
    getattr(p2, name)[idx] = x0 - h
    return (_loss(p1, cam, dldc, cull=cull)[0] - _loss(p2, cam, dldc, cull=cull)[0]) / (2 * h)


def _check_all(params, cam, dldc, cull=None, groups=("means", "scales", "quats", "opacity", "sh"), tol=2e-6):
    L, out = _loss(params, cam, dldc, cull=cull)
    mg = _margins_ok(params, cam, out)
    assert mg["decision"] > 1e-3 and mg["clamp"] > 1e-3 and mg["zgap"] > 1e-5 and mg["raw"] > 1e-3, mg
    assert mg["jac"] > 1e-3, mg
    grads, _ = oracle.backward_views(params, [cam], OPTS, [dldc], cull_mask=cull)
    for name in groups:
        g = grads[name]
        fd = np.zeros_like(g)
        for idx in np.ndindex(*g.shape):
            if name == "sh" and idx[0] >= (params.sh_degree + 1) ** 2:
                continue
            fd[idx] = _fd(params, cam, dldc, name, idx, cull=cull)
        err = np.linalg.norm(g - fd) / max(np.linalg.norm(fd), 1e-30)
        assert err < tol, (name, err)
        assert np.abs(g - fd).max() <= 1e-6 * max(np.abs(fd).max(), 1e-12) + 1e-9, name


@pytest.mark.parametrize("seed", [0, 1])
def test_parameter_gradients_match_central_differences(seed):
    sc = random_small_scene(seed + 20, n=8, spread=0.5, scale_lo=0.08, scale_hi=0.25, degree=3)
    cam = gs_inputs.look_at((0.4, -0.3, 3.0), (0, 0, 0), 28, 22, 55.0)
    dldc = gs_inputs.rng(seed + 40).normal(size=(28 * 22, 3))
    _check_all(oracle.Params.of(sc), cam, dldc)


def test_gradients_through_the_jacobian_clamp():
    # one Gaussian beyond 1.3 x tan(fov/2) to the side, large enough to reach the
    # image: its J uses the clamped ratio, so d/dt_x of J vanishes.
    cam = gs_inputs.look_at((0.0, 0.0, 3.0), (0, 0, 0), 32, 24, 55.0)
    g = gs_inputs.rng(5)
    sc = scene_from([[2.7, 0.1, 0.0], [0.1, 0.0, 0.2]], [[0.6, 0.5, 0.55], [0.15, 0.2, 0.1]],
                    [g.normal(size=4), g.normal(size=4)], [0.9, 0.6],
                    dc_rgb=[[0.7, 0.4, 0.2], [0.2, 0.6, 0.5]], degree=0)
    p = oracle.Params.of(sc)
    P = oracle.project(p, cam, OPTS)
    lim = OPTS.jac_clamp * cam.width / (2 * cam.fx)
    assert abs(P[0, F["TXTZ"]]) > lim + 0.05 and P[0, F["VALID"]] == 1 and P[0, F["TILES"]] > 0
    dldc = gs_inputs.rng(6).normal(size=(32 * 24, 3))
    _check_all(p, cam, dldc, groups=("means", "scales", "quats", "opacity"))


def test_cull_mask_gradients():
    sc = random_small_scene(31, n=6, spread=0.5, scale_lo=0.1, scale_hi=0.25, degree=1)
    cam = gs_inputs.look_at((0.2, 0.1, 3.0), (0, 0, 0), 24, 20, 55.0)
    cull = np.array([1, 0, 1, 1, 0, 1], dtype=np.uint8)
    dldc = gs_inputs.rng(7).normal(size=(24 * 20, 3))
    p = oracle.Params.of(sc)
    _check_all(p, cam, dldc, cull=cull, groups=("means", "opacity", "sh"))
    grads, _ = oracle.backward_views(p, [cam], OPTS, [dldc], cull_mask=cull)
    for k, g in grads.items():
        assert np.all(g[..., cull == 0] == 0)


@pytest.mark.parametrize("seed", [3, 4])
def test_render_backward_matches_differences_of_record_fields(seed):
    # stage-level: perturb the 2D record (u, v, conic, opacity, rgb) directly.
    sc = random_small_scene(seed, n=10, spread=0.5, scale_lo=0.05, scale_hi=0.25)
    cam = gs_inputs.look_at((0.3, 0.2, 3.2), (0, 0, 0), 30, 26, 55.0)
    p = oracle.Params.of(sc)
    proj = oracle.project(p, cam, OPTS)
    ordr = oracle.order(proj)
    dldc = gs_inputs.rng(seed + 9).normal(size=(30 * 26, 3))
    base = oracle.render(p, cam, proj, ordr, OPTS, accumulate=False)
    assert base["margin"][:, :2].min() > 1e-3 and base["margin"][:, 3].min() > 1e-3
    g2d = oracle.render_backward(p, cam, proj, ordr, OPTS, dldc)
    fields = [F["U"], F["V"], F["CA"], F["CB"], F["CC"], F["OPAC"], F["R"], F["G"], F["B"]]
    fd = np.zeros_like(g2d)
    for i in ordr:
        for j, fld in enumerate(fields):
            h = 1e-6 * max(1.0, abs(proj[i, fld]))
            a = proj.copy()
            a[i, fld] += h
            b = proj.copy()
            b[i, fld] -= h
            la = (oracle.render(p, cam, a, ordr, OPTS, accumulate=False)["color"] * dldc).sum()
            lb = (oracle.render(p, cam, b, ordr, OPTS, accumulate=False)["color"] * dldc).sum()
            fd[i, j] = (la - lb) / (2 * h)
    assert np.linalg.norm(g2d - fd) / np.linalg.norm(fd) < 1e-6
    assert np.abs(g2d - fd).max() < 1e-6 * np.abs(fd).max()


def test_single_gaussian_closed_form_gradients():
    # dC/dk00 = w Y00 and dC/do = T G rgb (T = 1 for the only Gaussian).
    f, z0, W, H = 32.0, 4.0, 32, 32
    cam = identity_camera(W, H, f, z0)
    sc = scene_from([0.1, -0.05, 0.0], [0.06, 0.05, 0.07], [0.9, 0.1, 0.2, -0.1], [0.6],
                    dc_rgb=[[0.3, 0.6, 0.9]])
    p = oracle.Params.of(sc)
    out = oracle.forward_view(p, cam, OPTS)
    P = out["proj"][0]
    pix = 17 * W + 16
    dldc = np.zeros((W * H, 3))
    dldc[pix, 0] = 1.0
    grads, _ = oracle.backward_views(p, [cam], OPTS, [dldc])
    dx, dy = 16.5 - P[F["U"]], 17.5 - P[F["V"]]
    G = math.exp(-0.5 * (P[F["CA"]] * dx * dx + 2 * P[F["CB"]] * dx * dy + P[F["CC"]] * dy * dy))
    w = float(np.float32(0.6)) * G
    assert out["color"][pix, 0] == pytest.approx(w * P[F["R"]], rel=1e-12)
    assert grads["sh"][0, 0, 0] == pytest.approx(w * 0.5 / math.sqrt(math.pi), rel=1e-12)
    assert grads["opacity"][0] == pytest.approx(G * P[F["R"]], rel=1e-12)
    assert grads["sh"][0, 1, 0] == 0 and grads["sh"][0, 2, 0] == 0


def test_active_mask_zeroes_rows_only():
    sc = random_small_scene(2, n=10)
    cam = gs_inputs.look_at((0.3, 0.2, 3.2), (0, 0, 0), 30, 26, 55.0)
    p = oracle.Params.of(sc)
    dldc = gs_inputs.rng(1).normal(size=(30 * 26, 3))
    full, _ = oracle.backward_views(p, [cam], OPTS, [dldc])
    act = gs_inputs.bernoulli_mask(10, 0.5, 3)
    masked, _ = oracle.backward_views(p, [cam], OPTS, [dldc], active=act)
    for k in full:
        assert np.array_equal(masked[k][..., act == 1], full[k][..., act == 1])
        assert np.all(masked[k][..., act == 0] == 0)
