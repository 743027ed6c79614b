"""Pins for the oracle's decision branches (test support for comparing a
float32 renderer with the FP64 definition of Eq. (1)-(2)).

Eq. (1) takes discrete decisions per pair: skip (alpha below alpha_min), stop
(transmittance would fall below t_min) and, for Eq. (2), whether a weight
beats the best so far.  Where a decision's operands lie within float32
rounding of the threshold, a float32 renderer may take the other branch; the
oracle then enumerates every branch.  These pins build scenes whose decisions
sit on a threshold by construction and check each branch against the closed
form of Eq. (1) with that decision taken either way.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import F
from tests.oracle_scenes import identity_camera, random_small_scene, scene_from

OPTS = oracle.Opts()
AMB = (2e-5, 2e-3, 1e-4)  # alpha, stop, argmax widths
W = H = 32
FOCAL, Z0 = 32.0, 4.0
PX, PY = 10, 7
CAM = identity_camera(W, H, FOCAL, Z0)


def _on_pixel_ray(z):
    """World (x, y, z) that projects to the centre of pixel (PX, PY)."""
    return [(PX + 0.5 - W / 2) * (z + Z0) / FOCAL, (PY + 0.5 - H / 2) * (z + Z0) / FOCAL, z]


def _setup(sc):
    p = oracle.Params.of(sc)
    proj = oracle.project(p, CAM, OPTS)
    return p, proj, oracle.order(proj)


def _branches(sc, pixels=((PX, PY),)):
    p, proj, ordr = _setup(sc)
    pix = np.array(pixels, dtype=np.int32)
    return oracle.branches(p, CAM, proj, ordr, OPTS, pix, AMB), p, proj, ordr, pix


def _alpha(P, x, y):
    dx, dy = x + 0.5 - P[F["U"]], y + 0.5 - P[F["V"]]
    q = P[F["CA"]] * dx * dx + 2 * P[F["CB"]] * dx * dy + P[F["CC"]] * dy * dy
    return min(OPTS.alpha_max, P[F["OPAC"]] * np.exp(-0.5 * q))


def _rgb(P):
    return np.array([P[F["R"]], P[F["G"]], P[F["B"]]])


def test_zero_flips_reproduce_the_definition():
    sc = random_small_scene(3, n=40)
    p, proj, ordr = _setup(sc)
    plain = oracle.render(p, CAM, proj, ordr, OPTS)
    flipped = oracle.render(p, CAM, proj, ordr, OPTS, amb=AMB, flips=np.zeros(W * H, dtype=np.uint32))
    for k in ("color", "t_final", "n_contrib", "imax", "depth", "hit", "importance", "wmax", "area"):
        assert np.array_equal(plain[k], flipped[k]), k
    g = np.random.default_rng(0).normal(size=(W * H, 3))
    assert np.array_equal(oracle.render_backward(p, CAM, proj, ordr, OPTS, g),
                          oracle.render_backward(p, CAM, proj, ordr, OPTS, g, amb=AMB,
                                                 flips=np.zeros(W * H, dtype=np.uint32)))


def test_skip_decision_on_the_threshold():
    # opacity a millionth above alpha_min, centred on the pixel: included by the
    # definition, skipped on the other branch
    o = float(np.float32(OPTS.alpha_min * (1 + 1e-6)))
    assert o > OPTS.alpha_min
    sc = scene_from([_on_pixel_ray(0.0)], [[0.05] * 3], [[1, 0, 0, 0]], [o], dc_rgb=[[0.2, 0.6, 0.9]])
    b, p, proj, ordr, pix = _branches(sc)
    assert b["complete"][0] and b["count"][0] == 2
    a = _alpha(proj[0], PX, PY)
    assert abs(a - OPTS.alpha_min) / OPTS.alpha_min < AMB[0]
    by_n = {int(b["n_contrib"][0, j]): j for j in range(2)}
    assert set(by_n) == {0, 1}
    inc, skp = by_n[1], by_n[0]
    assert b["flips"][0, inc] == 0  # the definition's own decision is branch 0
    assert np.allclose(b["color"][0, inc], a * _rgb(proj[0]), rtol=1e-12)
    assert b["t_final"][0, inc] == pytest.approx(1 - a, rel=1e-14)
    assert b["imax"][0, inc] == 0 and b["imax"][0, skp] == -1
    assert np.all(b["color"][0, skp] == 0) and b["t_final"][0, skp] == 1.0 and b["depth"][0, skp] == 0
    # the backward follows the branch: the skipped pair passes no gradient
    g = np.ones((1, 3))
    g_inc = oracle.render_backward(p, CAM, proj, ordr, OPTS, g, pixels=pix, amb=AMB,
                                   flips=np.array([b["flips"][0, inc]], dtype=np.uint32))
    g_skp = oracle.render_backward(p, CAM, proj, ordr, OPTS, g, pixels=pix, amb=AMB,
                                   flips=np.array([b["flips"][0, skp]], dtype=np.uint32))
    assert np.all(g_skp == 0) and np.allclose(g_inc[0, 6:], a)
    # pixels away from the centre are far below alpha_min: a single branch
    b2, *_ = _branches(sc, pixels=((PX + 2, PY), (0, 0)))
    assert list(b2["count"]) == [1, 1] and list(b2["n_contrib"][:, 0]) == [0, 0]


def test_stop_decision_on_the_threshold():
    # two clamped Gaussians (alpha = 0.99) on one ray: (1 - 0.99)^2 lies 2e-6
    # below t_min in float32 constants, so the definition stops before the
    # second; the other branch includes it
    c1, c2 = [0.9, 0.1, 0.2], [0.1, 0.8, 0.3]
    sc = scene_from([_on_pixel_ray(0.0), _on_pixel_ray(1.0)], [[0.05] * 3] * 2, [[1, 0, 0, 0]] * 2,
                    [0.995, 0.995], dc_rgb=[c1, c2])
    b, p, proj, ordr, pix = _branches(sc)
    assert b["complete"][0] and b["count"][0] == 2
    am = OPTS.alpha_max
    assert _alpha(proj[0], PX, PY) == am and _alpha(proj[1], PX, PY) == am
    T1 = 1 - am
    assert T1 * (1 - am) < OPTS.t_min and abs(T1 * (1 - am) - OPTS.t_min) / OPTS.t_min < AMB[1]
    by_n = {int(b["n_contrib"][0, j]): j for j in range(2)}
    assert set(by_n) == {1, 2}
    stop, inc = by_n[1], by_n[2]
    assert b["flips"][0, stop] == 0
    assert np.allclose(b["color"][0, stop], am * _rgb(proj[0]), rtol=1e-14)
    assert b["t_final"][0, stop] == pytest.approx(T1, rel=1e-14)
    assert np.allclose(b["color"][0, inc], am * _rgb(proj[0]) + T1 * am * _rgb(proj[1]), rtol=1e-14)
    assert b["t_final"][0, inc] == pytest.approx(T1 * (1 - am), rel=1e-14)
    assert b["t_final"][0, inc] < OPTS.t_min  # the branch that continues passes the stop
    assert b["imax"][0, stop] == 0 and b["imax"][0, inc] == 0  # 0.99 beats 0.0099
    g = np.ones((1, 3))
    g_stop = oracle.render_backward(p, CAM, proj, ordr, OPTS, g, pixels=pix, amb=AMB,
                                    flips=np.array([b["flips"][0, stop]], dtype=np.uint32))
    g_inc = oracle.render_backward(p, CAM, proj, ordr, OPTS, g, pixels=pix, amb=AMB,
                                   flips=np.array([b["flips"][0, inc]], dtype=np.uint32))
    assert np.all(g_stop[1] == 0) and np.allclose(g_inc[1, 6:], T1 * am)


def test_argmax_decision_on_a_tie():
    # w1 = a1 and w2 = (1 - a1) a2 with a2 = a1 / (1 - a1): equal up to float32
    # rounding of the opacities, so either Gaussian may be the rendered index
    a1 = 0.3
    sc = scene_from([_on_pixel_ray(0.0), _on_pixel_ray(1.5)], [[0.05] * 3] * 2, [[1, 0, 0, 0]] * 2,
                    [a1, a1 / (1 - a1)], dc_rgb=[[0.5, 0.5, 0.5], [0.3, 0.2, 0.1]])
    b, p, proj, ordr, pix = _branches(sc)
    assert b["complete"][0] and b["count"][0] == 2
    w1 = _alpha(proj[0], PX, PY)
    w2 = (1 - w1) * _alpha(proj[1], PX, PY)
    assert abs(w1 - w2) / max(w1, w2) < AMB[2]
    assert sorted(b["imax"][0, :2].tolist()) == [0, 1]
    # the tie moves the rendered index (and its depth), not the colour
    assert np.array_equal(b["color"][0, 0], b["color"][0, 1]) and b["n_contrib"][0, 0] == b["n_contrib"][0, 1] == 2
    j1 = int(np.nonzero(b["imax"][0, :2] == 1)[0][0])
    j0 = 1 - j1
    assert b["depth"][0, j0] == pytest.approx(proj[0, F["Z"]], rel=1e-9)
    assert b["depth"][0, j1] == pytest.approx(proj[1, F["Z"]], rel=1e-9)
    plain = oracle.render(p, CAM, proj, ordr, OPTS, pixels=pix, accumulate=False)
    assert plain["imax"][0] == (1 if w2 > w1 else 0) == b["imax"][0, 0]


def test_every_combination_of_independent_decisions():
    # three faint Gaussians on one ray, each a millionth above alpha_min: their
    # skip decisions do not depend on each other, so all 2^3 subsets are branches
    o = float(np.float32(OPTS.alpha_min * (1 + 1e-6)))
    cols = [[0.9, 0.1, 0.1], [0.1, 0.9, 0.1], [0.1, 0.1, 0.9]]
    sc = scene_from([_on_pixel_ray(z) for z in (0.0, 0.7, 1.4)], [[0.05] * 3] * 3, [[1, 0, 0, 0]] * 3, [o] * 3,
                    dc_rgb=cols)
    b, p, proj, ordr, pix = _branches(sc)
    assert b["complete"][0] and b["count"][0] == 8
    a = [_alpha(proj[k], PX, PY) for k in range(3)]
    want = []
    for sub in itertools.product((0, 1), repeat=3):
        T, C = 1.0, np.zeros(3)
        for k in range(3):
            if sub[k]:
                C = C + T * a[k] * _rgb(proj[k])
                T *= 1 - a[k]
        want.append((sum(sub), C, T))
    got = [(int(b["n_contrib"][0, j]), b["color"][0, j], b["t_final"][0, j]) for j in range(8)]
    for n_, C, T in want:
        assert sum(1 for g in got if g[0] == n_ and np.allclose(g[1], C, rtol=1e-12, atol=0)
                   and abs(g[2] - T) <= 1e-14) == 1
    assert len(set(b["flips"][0, :8].tolist())) == 8
    # a branch cap below the count is reported, not silently truncated
    p_, proj_, ordr_ = _setup(sc)
    capped = oracle.branches(p_, CAM, proj_, ordr_, OPTS, pix, AMB, max_branches=4)
    assert capped["count"][0] == 4 and not capped["complete"][0]


def test_no_ambiguity_means_one_branch():
    sc = random_small_scene(5, n=30)
    p, proj, ordr = _setup(sc)
    plain = oracle.render(p, CAM, proj, ordr, OPTS, accumulate=False)
    m = plain["margin"]
    clear = np.nonzero((m[:, 0] >= AMB[0]) & (m[:, 1] >= AMB[1]) & (m[:, 2] >= AMB[2]))[0][:50]
    pix = np.stack([clear % W, clear // W], 1).astype(np.int32)
    b = oracle.branches(p, CAM, proj, ordr, OPTS, pix, AMB)
    assert np.all(b["count"] == 1)
    assert np.array_equal(b["color"][:, 0], plain["color"][clear])
    assert np.array_equal(b["imax"][:, 0], plain["imax"][clear])


def test_tiled_backward_equals_untiled():
    # restricting each pixel to its tile's list removes only pairs below
    # alpha_min, so the gradient is the same (tiled == untiled for Eq. (1)'s
    # derivative as for the forward)
    sc = random_small_scene(11, n=60, spread=0.9, scale_lo=0.03, scale_hi=0.2)
    cam = identity_camera(48, 40, 40.0, 3.0)
    p = oracle.Params.of(sc)
    proj = oracle.project(p, cam, OPTS)
    ordr = oracle.order(proj)
    tx, ty, base, total = oracle.view_layout([cam])
    _, vals, ranges = oracle.bin(oracle.tile_rects(proj), oracle.zbits(proj), 1, sc.n, base, tx, total)
    g = np.random.default_rng(1).normal(size=(48 * 40, 3))
    full = oracle.render_backward(p, cam, proj, ordr, OPTS, g)
    tiled = oracle.render_backward(p, cam, proj, ordr, OPTS, g, tiles=(vals, ranges))
    assert np.abs(full).max() > 0
    assert np.allclose(tiled, full, rtol=1e-12, atol=1e-15)


def test_float32_weight_error_within_bound():
    """The oracle's first-order bound of a float32 renderer's error in each
    weight w = alpha T holds for an emulated float32 compositing of the same
    pairs (alpha = exp2 of a float32 exponent, float32 transmittance product),
    and is not vacuous.  Pixels are taken whole: one pixel at a time, so the
    per-Gaussian bound is the per-pair bound."""
    sc = random_small_scene(21, n=80, spread=0.5, scale_lo=0.05, scale_hi=0.25)
    sc.opacity[:] = np.linspace(0.3, 0.995, sc.n).astype(np.float32)
    p, proj, ordr = _setup(sc)
    f32 = np.float32
    l2e = 1.4426950408889634
    checked, ratios = 0, []
    for (x, y) in [(x, y) for y in range(6, 26, 3) for x in range(6, 26, 3)]:
        pix = np.array([[x, y]], dtype=np.int32)
        o = oracle.render(p, CAM, proj, ordr, OPTS, pixels=pix, accumulate=True)
        T32 = f32(1.0)
        for g in ordr:
            P = proj[g]
            dx, dy = f32(x + 0.5 - P[F["U"]]), f32(y + 0.5 - P[F["V"]])
            A, B, C = f32(0.5 * l2e * P[F["CA"]]), f32(l2e * P[F["CB"]]), f32(0.5 * l2e * P[F["CC"]])
            ee = f32(np.log2(P[F["OPAC"]])) - (A * dx * dx + B * dx * dy + C * dy * dy)
            a32 = min(f32(OPTS.alpha_max), np.exp2(ee, dtype=np.float32))
            Tn = T32 * (f32(1.0) - a32)
            inc32 = a32 >= f32(OPTS.alpha_min) and Tn >= f32(OPTS.t_min)
            if inc32 != (o["acc_tol"][g, 2] == 1):
                break  # the float32 walk left the oracle's decisions: not this pin's case
            if a32 >= f32(OPTS.alpha_min) and Tn < f32(OPTS.t_min):
                break
            if not inc32:
                continue
            w32 = float(a32 * T32)
            T32 = Tn
            w64, tol = o["importance"][g], o["acc_tol"][g, 0]
            assert abs(w32 - w64) <= tol, (x, y, g, w32, w64, tol)
            ratios.append(abs(w32 - w64) / tol)
            checked += 1
    assert checked > 100
    assert max(ratios) > 1e-3  # the bound is tight enough to matter
    # a clamped alpha carries no error of its own: only the product's rounding
    sc1 = scene_from([_on_pixel_ray(0.0)], [[0.05] * 3], [[1, 0, 0, 0]], [0.995], dc_rgb=[[0.5] * 3])
    p1, proj1, ordr1 = _setup(sc1)
    o1 = oracle.render(p1, CAM, proj1, ordr1, OPTS, pixels=np.array([[PX, PY]], dtype=np.int32), accumulate=True)
    assert o1["acc_tol"][0, 0] == pytest.approx(OPTS.alpha_max * 2.0 ** -24, rel=1e-12)
    assert o1["acc_tol"][0, 2] == 1
