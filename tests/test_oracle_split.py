"""Pins of the oracle's 3DGS density control: the clone/split selection and the
split into two children drawn from the parent (Sec. 3.2; the blur split of
Sec. 4.1 hands its Gaussians to the same split).  Rotation conventions are
pinned against scipy's quaternion rotation and closed-form rotations, the
children's spread against the parent covariance by Monte Carlo."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import gs_inputs
import oracle
from gs_inputs import uniform_cube_scene


def _params(n, seed=5):
    return oracle.Params.of(uniform_cube_scene(n, seed=seed))


def test_split_identity_rotation_closed_form():
    p = _params(3)
    p.quats[:] = 0.0
    p.quats[0] = 2.5  # unnormalised identity
    z = gs_inputs.rng(1).normal(size=(2, 3, 3))
    out = oracle.split(p, np.array([0, 1, 0]), z)
    assert out.n == 4
    for c in range(2):
        d = 2 + c
        np.testing.assert_array_equal(out.means[:, d], p.means[:, 1] + p.scales[:, 1] * z[c, :, 1])
        np.testing.assert_array_equal(out.scales[:, d], p.scales[:, 1] / 1.6)


def test_split_quarter_turn_about_z():
    # q = (cos 45, 0, 0, sin 45) turns x into y; the child offset of z = e_x is
    # therefore s_x e_y, and of z = e_y it is -s_y e_x
    p = _params(1)
    p.means[:, 0] = (1.0, -2.0, 0.5)
    p.scales[:, 0] = (2.0, 0.5, 0.1)
    p.quats[:, 0] = (math.cos(math.pi / 4), 0.0, 0.0, math.sin(math.pi / 4))
    z = np.zeros((2, 3, 1))
    z[0, 0, 0] = 1.0
    z[1, 1, 0] = 1.0
    out = oracle.split(p, np.array([1]), z)
    np.testing.assert_allclose(out.means[:, 0], (1.0, 0.0, 0.5), atol=1e-15)
    np.testing.assert_allclose(out.means[:, 1], (0.5, -2.0, 0.5), atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_split_rotation_matches_scipy(seed):
    g = gs_inputs.rng(seed)
    n = 16
    p = _params(n, seed)
    z = g.normal(size=(2, 3, n))
    out = oracle.split(p, np.ones(n), z)
    q = p.quats.T  # (w, x, y, z) rows
    R = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], 1)).as_matrix()
    for c in range(2):
        off = np.einsum("nij,nj->ni", R, (p.scales * z[c]).T)
        np.testing.assert_allclose(out.means[:, 2 * np.arange(n) + c].T, p.means.T + off, rtol=0, atol=1e-12)


def test_split_children_spread_like_the_parent():
    # children are draws from N(p, R S^2 R^T): their sample covariance over many
    # draws approaches the parent's covariance (a transposed R would not)
    g = gs_inputs.rng(7)
    p = _params(1, 11)
    p.scales[:, 0] = (0.3, 0.05, 0.01)
    p.quats[:, 0] = (0.7, 0.2, -0.5, 0.4)
    k = 40000
    many = oracle.Params(np.repeat(p.means, k, 1), np.repeat(p.scales, k, 1), np.repeat(p.quats, k, 1),
                         np.repeat(p.opacity, k), np.repeat(p.sh, k, 2), p.sh_degree)
    z = g.normal(size=(2, 3, k))
    out = oracle.split(many, np.ones(k), z)
    d = out.means - p.means
    cov = d @ d.T / d.shape[1]
    q = p.quats[:, 0] / np.linalg.norm(p.quats[:, 0])
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    sigma = R @ np.diag(p.scales[:, 0] ** 2) @ R.T
    np.testing.assert_allclose(cov, sigma, atol=0.03 * sigma.max())
    wrong = R.T @ np.diag(p.scales[:, 0] ** 2) @ R
    assert np.abs(cov - wrong).max() > 0.1 * sigma.max()


def test_split_layout_and_copies():
    n = 9
    p = _params(n)
    sel = np.array([0, 1, 1, 0, 0, 1, 0, 0, 1], dtype=np.uint8)
    z = gs_inputs.rng(3).normal(size=(2, 3, n))
    out = oracle.split(p, sel, z)
    keep = np.flatnonzero(sel == 0)
    chosen = np.flatnonzero(sel)
    assert out.n == n + len(chosen)
    np.testing.assert_array_equal(out.means[:, :len(keep)], p.means[:, keep])
    np.testing.assert_array_equal(out.scales[:, :len(keep)], p.scales[:, keep])
    src = np.concatenate([keep, np.repeat(chosen, 2)])
    np.testing.assert_array_equal(out.quats, p.quats[:, src])
    np.testing.assert_array_equal(out.opacity, p.opacity[src])
    np.testing.assert_array_equal(out.sh, p.sh[:, :, src])


def test_split_zero_draws_and_zero_quaternion():
    p = _params(2)
    p.quats[:, 1] = 0.0
    z = np.zeros((2, 3, 2))
    out = oracle.split(p, np.ones(2), z)
    np.testing.assert_array_equal(out.means, p.means[:, [0, 0, 1, 1]])
    z[:, :, 1] = 1.0  # zero quaternion: identity rotation
    out = oracle.split(p, np.ones(2), z)
    np.testing.assert_array_equal(out.means[:, 2], p.means[:, 1] + p.scales[:, 1])


def test_split_nothing_selected_and_empty():
    p = _params(5)
    out = oracle.split(p, np.zeros(5), np.zeros((2, 3, 5)))
    np.testing.assert_array_equal(out.means, p.means)
    np.testing.assert_array_equal(out.sh, p.sh)
    e = oracle.split(_params(0), np.zeros(0), np.zeros((2, 3, 0)))
    assert e.n == 0


def test_densify_select_boundaries():
    # mean gradient exactly at the threshold is selected; largest scale exactly
    # at the scale threshold clones, above it splits; never-seen rows are idle
    norm_sum = np.array([3.0, 3.0, 2.9, 5.0, 0.0, 4.0])
    count = np.array([2, 2, 2, 2, 0, 1])
    scales = np.array([[0.1, 0.1, 0.1, 0.01, 1.0, 0.2],
                       [0.2, 0.30000001, 0.1, 0.01, 1.0, 0.2],
                       [0.1, 0.1, 0.1, 0.5, 1.0, 0.3]])
    clone, split = oracle.densify_select(norm_sum, count, scales, 1.5, 0.3)
    np.testing.assert_array_equal(clone, [True, False, False, False, False, True])
    np.testing.assert_array_equal(split, [False, True, False, True, False, False])


def test_densify_select_uses_the_largest_scale():
    # mean scale below, largest above the threshold: split, not clone
    scales = np.array([[0.01], [0.01], [0.9]])
    clone, split = oracle.densify_select([1.0], [1], scales, 0.5, 0.4)
    assert split[0] and not clone[0]
