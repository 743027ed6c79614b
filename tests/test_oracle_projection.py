"""Pins for the oracle's projection (EWA covariance, SH colour, extents).

Each test ties the oracle to something other than itself: scipy's spherical
harmonics and rotations, numerical quadrature, Monte-Carlo projection of
samples, closed forms on special configurations, brute-force enumeration.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import gs_inputs
import oracle
from oracle import F
from tests.oracle_scenes import identity_camera, scene_from

OPTS = oracle.Opts()


def _real_sh_scipy(l, m, d):
    """Real SH without Condon-Shortley phase from scipy's complex SH (which has it)."""
    from scipy import special
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    if hasattr(special, "sph_harm_y"):
        Ylm = special.sph_harm_y(l, abs(m), theta, phi)
    else:  # older scipy: sph_harm(m, l, azimuth, polar)
        Ylm = special.sph_harm(abs(m), l, phi, theta)
    if m > 0:
        return math.sqrt(2) * (-1) ** m * Ylm.real
    if m < 0:
        return math.sqrt(2) * (-1) ** m * Ylm.imag
    return Ylm.real


def test_sh_basis_matches_scipy():
    g = gs_inputs.rng(11)
    for _ in range(25):
        d = g.normal(size=3)
        d /= np.linalg.norm(d)
        Y = oracle.sh_basis(d, 3)
        for l in range(4):
            for m in range(-l, l + 1):
                assert Y[l * l + l + m] == pytest.approx(_real_sh_scipy(l, m, d), abs=1e-12)


def test_sh_basis_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform azimuth integrates degree-6 products exactly.
    xs, ws = np.polynomial.legendre.leggauss(12)
    nphi = 24
    G = np.zeros((16, 16))
    for ct, wt in zip(xs, ws):
        st = math.sqrt(1 - ct * ct)
        for k in range(nphi):
            ph = 2 * math.pi * k / nphi
            Y = oracle.sh_basis(np.array([st * math.cos(ph), st * math.sin(ph), ct]), 3)
            G += wt * (2 * math.pi / nphi) * np.outer(Y, Y)
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_sh_basis_degree_truncation():
    d = np.array([0.3, -0.4, math.sqrt(1 - 0.25)])
    Y3 = oracle.sh_basis(d, 3)
    for deg in range(4):
        Y = oracle.sh_basis(d, deg)
        k = (deg + 1) ** 2
        assert np.array_equal(Y[:k], Y3[:k]) and np.all(Y[k:] == 0)


def test_sh_gradient_by_finite_differences():
    g = gs_inputs.rng(12)
    for _ in range(10):
        d = g.normal(size=3)
        dY = oracle.sh_basis_grad(d, 3)
        h = 1e-6
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            fd = (oracle.sh_basis(d + e, 3) - oracle.sh_basis(d - e, 3)) / (2 * h)
            assert np.allclose(fd, dY[:, c], atol=1e-8)


def _params(sc):
    return oracle.Params.of(sc)


@pytest.mark.parametrize("qseed", [0, 1, 2])
def test_isotropic_on_axis_closed_form(qseed):
    # Sigma' = (f s / z)^2 I + lowpass I, independent of the rotation.
    f, z0, s = 40.0, 5.0, 0.07
    cam = identity_camera(64, 48, f, z0)
    q = gs_inputs.rng(qseed).normal(size=4)
    sc = scene_from([0, 0, 0], [s, s, s], q, [0.7], dc_rgb=[[0.2, 0.4, 0.6]])
    P = oracle.project(_params(sc), cam, OPTS)[0]
    s_f, f_f, z_f = float(np.float32(s)), float(np.float32(f)), float(np.float32(z0))
    var = (f_f * s_f / z_f) ** 2 + OPTS.lowpass
    assert P[F["VALID"]] == 1
    assert P[F["U"]] == pytest.approx(32.0, abs=1e-12) and P[F["V"]] == pytest.approx(24.0, abs=1e-12)
    assert P[F["S00"]] == pytest.approx(var, rel=1e-12) and P[F["S11"]] == pytest.approx(var, rel=1e-12)
    assert abs(P[F["S01"]]) < 1e-12 * var
    assert P[F["CA"]] == pytest.approx(1 / var, rel=1e-12) and P[F["CC"]] == pytest.approx(1 / var, rel=1e-12)
    assert P[F["Z"]] == pytest.approx(z_f, rel=1e-15)
    assert tuple(P[[F["R"], F["G"], F["B"]]]) == pytest.approx((0.2, 0.4, 0.6), abs=1e-7)


@pytest.mark.parametrize("quat,swap", [((1, 0, 0, 0), (0, 1)),
                                       ((math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)), (1, 0)),
                                       ((-math.cos(math.pi / 4), 0, 0, -math.sin(math.pi / 4)), (1, 0)),
                                       ((math.cos(math.pi / 4), math.sin(math.pi / 4), 0, 0), (0, 2))])
def test_axis_aligned_rotations_closed_form(quat, swap):
    # identity rotation keeps (sx, sy); 90 deg about z swaps them; -q == q;
    # 90 deg about x maps the z axis into image y.
    f, z0 = 50.0, 4.0
    s = np.array([0.05, 0.11, 0.23], dtype=np.float32)
    cam = identity_camera(80, 80, f, z0)
    sc = scene_from([0, 0, 0], s, quat, [0.5], dc_rgb=[[0.5, 0.5, 0.5]])
    P = oracle.project(_params(sc), cam, OPTS)[0]
    sx, sy = float(s[swap[0]]), float(s[swap[1]])
    fz = float(np.float32(f)) / float(np.float32(z0))
    assert P[F["S00"]] == pytest.approx((fz * sx) ** 2 + OPTS.lowpass, rel=1e-6)
    assert P[F["S11"]] == pytest.approx((fz * sy) ** 2 + OPTS.lowpass, rel=1e-6)
    assert abs(P[F["S01"]]) < 1e-6


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_ewa_covariance_matches_monte_carlo(seed):
    # Sigma' - lowpass is the covariance of samples of N(p, Sigma) pushed through
    # the pinhole, to first order in sigma / z.
    g = gs_inputs.rng(seed)
    eye = g.normal(size=3)
    eye = 5.0 * eye / np.linalg.norm(eye)
    cam = gs_inputs.look_at(eye, (0, 0, 0), 640, 480, 60.0)
    p = g.uniform(-0.8, 0.8, size=3)
    s = np.exp(g.normal(-4.5, 0.4, size=3))
    q = g.normal(size=4)
    q /= np.linalg.norm(q)
    sc = scene_from(p, s, q, [0.6], dc_rgb=[[0.5, 0.5, 0.5]])
    P = oracle.project(_params(sc), cam, OPTS)[0]
    # independent covariance construction via scipy (quaternion order x, y, z, w)
    pf = sc.means[:, 0].astype(np.float64)
    sf = sc.scales[:, 0].astype(np.float64)
    qf = sc.quats[:, 0].astype(np.float64)
    Rq = Rotation.from_quat([qf[1], qf[2], qf[3], qf[0]]).as_matrix()
    Sig = Rq @ np.diag(sf ** 2) @ Rq.T
    M = 1_500_000
    X = g.multivariate_normal(pf, Sig, size=M)
    Rc = cam.R.astype(np.float64)
    tc = cam.t.astype(np.float64)
    Tc = X @ Rc.T + tc
    uv = np.stack([cam.fx * Tc[:, 0] / Tc[:, 2] + cam.cx, cam.fy * Tc[:, 1] / Tc[:, 2] + cam.cy], axis=1)
    emp = np.cov(uv.T)
    ewa = np.array([[P[F["S00"]] - OPTS.lowpass, P[F["S01"]]], [P[F["S01"]], P[F["S11"]] - OPTS.lowpass]])
    scale = np.linalg.eigvalsh(ewa).max()
    assert np.abs(emp - ewa).max() < 1e-2 * scale
    assert np.abs(uv.mean(axis=0) - np.array([P[F["U"]], P[F["V"]]])).max() < 3e-3 * math.sqrt(scale) + 1e-4


def test_extent_is_the_ellipse_bounding_box():
    g = gs_inputs.rng(7)
    cam = gs_inputs.look_at((1.0, 2.0, 6.0), (0, 0, 0), 200, 150, 50.0)
    for _ in range(5):
        p = g.uniform(-0.5, 0.5, size=3)
        s = np.exp(g.normal(-2.5, 0.5, size=3))
        q = g.normal(size=4)
        o = g.uniform(0.05, 0.95)
        P = oracle.project(_params(scene_from(p, s, q, [o], dc_rgb=[[0.5, 0.5, 0.5]])), cam, OPTS)[0]
        S = np.array([[P[F["S00"]], P[F["S01"]]], [P[F["S01"]], P[F["S11"]]]])
        L = np.linalg.cholesky(S)
        o32 = float(np.float32(o))
        k = 2 * math.log(o32 / OPTS.alpha_min)
        t = np.linspace(0, 2 * math.pi, 200001)
        bnd = math.sqrt(k) * (L @ np.stack([np.cos(t), np.sin(t)]))
        assert np.abs(bnd[0]).max() == pytest.approx(P[F["RX"]], rel=1e-9)
        assert np.abs(bnd[1]).max() == pytest.approx(P[F["RY"]], rel=1e-9)
        # alpha on the boundary is exactly the skip threshold
        K = np.linalg.inv(S)
        qv = np.einsum("ij,ik,kj->j", bnd[:, ::5000], K, bnd[:, ::5000])
        assert np.allclose(o32 * np.exp(-0.5 * qv), OPTS.alpha_min, rtol=1e-9)


def test_pixel_box_matches_enumeration():
    g = gs_inputs.rng(8)
    W, H = 97, 61
    cam = gs_inputs.look_at((0.0, 0.5, 4.0), (0, 0, 0), W, H, 60.0)
    sc = gs_inputs.uniform_cube_scene(300, 9, half=1.5, log_scale_mu=-2.5)
    proj = oracle.project(_params(sc), cam, OPTS)
    xs = np.arange(W) + 0.5
    ys = np.arange(H) + 0.5
    for P in proj:
        if P[F["VALID"]] == 0:
            continue
        inx = np.nonzero(np.abs(xs - P[F["U"]]) <= P[F["RX"]])[0]
        iny = np.nonzero(np.abs(ys - P[F["V"]]) <= P[F["RY"]])[0]
        if len(inx) == 0 or len(iny) == 0:
            assert P[F["XLO"]] > P[F["XHI"]] or P[F["YLO"]] > P[F["YHI"]]
            assert P[F["TILES"]] == 0
            continue
        assert (P[F["XLO"]], P[F["XHI"]], P[F["YLO"]], P[F["YHI"]]) == (inx[0], inx[-1], iny[0], iny[-1])
        ntx = inx[-1] // 16 - inx[0] // 16 + 1
        nty = iny[-1] // 16 - iny[0] // 16 + 1
        assert P[F["TILES"]] == ntx * nty


def test_invalid_records():
    cam = identity_camera(32, 32, 30.0, 3.0)
    means = [[0, 0, 0], [0, 0, -2.9], [0, 0, 0], [0, 0, 0], [0, 0, 0]]
    quats = [[1, 0, 0, 0], [1, 0, 0, 0], [0, 0, 0, 0], [1, 0, 0, 0], [1, 0, 0, 0]]
    opac = [0.5, 0.5, 0.5, 0.003, 0.5]
    sc = scene_from(means, [[0.1] * 3] * 5, quats, opac, dc_rgb=[[0.5] * 3] * 5)
    mask = np.array([1, 1, 1, 1, 0], dtype=np.uint8)
    proj = oracle.project(_params(sc), cam, OPTS, cull_mask=mask)
    # valid / behind the near plane / zero quaternion / opacity below 1/255 / culled
    assert list(proj[:, F["VALID"]]) == [1, 0, 0, 0, 0]
    assert list(proj[:, F["TILES"]]) == [4, 0, 0, 0, 0]


def test_colour_clamps_at_zero():
    cam = identity_camera(32, 32, 30.0, 3.0)
    sc = scene_from([0, 0, 0], [0.1] * 3, [1, 0, 0, 0], [0.5], dc_rgb=[[-0.3, 0.0, 1.7]])
    P = oracle.project(_params(sc), cam, OPTS)[0]
    assert P[F["R"]] == 0 and P[F["RAW_R"]] == pytest.approx(-0.3, abs=1e-7)
    assert P[F["B"]] == pytest.approx(1.7, abs=1e-6)


def test_params_of_slices_and_strided_arrays():
    """A Params built from column slices of another projects like the slice of
    the whole projection (the planes are copied contiguous); a strided array
    handed to the C oracle directly is refused rather than misread."""
    wl = gs_inputs.small_cube(seed=5, n=3000, width=112, height=96)
    p = oracle.Params.of(wl.scene)
    cam, opts = wl.cameras[0], oracle.Opts()
    full = oracle.project(p, cam, opts)
    sl = slice(1000, 2000)
    sub = oracle.Params(p.means[:, sl], p.scales[:, sl], p.quats[:, sl], p.opacity[sl], p.sh[:, :, sl], p.sh_degree)
    assert np.array_equal(oracle.project(sub, cam, opts), full[sl])
    with pytest.raises(ValueError):
        oracle._p(p.means[:, sl])
