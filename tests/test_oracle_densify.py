"""Pins for the oracle's densification and pruning criteria (Sec. 5.1, Sec. 5.2, Eq. (3)).

The quantile is pinned to numpy's linear-interpolation quantile; the clone is pinned
to what it is for: two copies at one centre must composite to the original peak
opacity, and the integral of the composite opacity along any line through the
centre must equal the original's (checked by quadrature, not by the closed form).
"""
import math

import numpy as np
import pytest

import oracle
import gs_inputs
from gs_inputs import uniform_cube_scene

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("q", [0.0, 0.01, 0.37, 0.5, 0.99, 1.0])
def test_quantile_matches_numpy(seed, q):
    rng = np.random.default_rng(seed)
    v = rng.exponential(size=1 + 97 * seed)
    mask = rng.random(v.shape[0]) < 0.6
    mask[0] = True
    assert oracle.quantile(v, q) == pytest.approx(np.quantile(v, q), rel=1e-14, abs=1e-300)
    assert oracle.quantile(v, q, mask) == pytest.approx(np.quantile(v[mask], q), rel=1e-14, abs=1e-300)


def test_quantile_empty_is_nan():
    assert math.isnan(oracle.quantile(np.zeros(0), 0.5))
    assert math.isnan(oracle.quantile(np.ones(4), 0.5, np.zeros(4, np.uint8)))


def test_quantile_ties_and_extremes():
    v = np.array([3.0, 1.0, 1.0, 1.0, 2.0])
    assert oracle.quantile(v, 0.0) == 1.0
    assert oracle.quantile(v, 1.0) == 3.0
    assert oracle.quantile(v, 0.5) == 1.0
    assert oracle.quantile(v, 0.875) == pytest.approx(2.5)


VALUE, MASS = oracle.THRESHOLD_VALUE, oracle.THRESHOLD_MASS


def test_visibility_keeps_top_fraction():
    rng = np.random.default_rng(5)
    imp = rng.lognormal(size=10000)
    imp[rng.random(imp.shape[0]) < 0.3] = 0.0        # non-contributors
    vis, tau, _ = oracle.visibility(imp, mode=VALUE)
    pos = imp[imp > 0]
    assert tau == pytest.approx(np.quantile(pos, 0.01))
    # strictly above the 1 % quantile: 99 % of contributors (up to ties / interpolation)
    assert abs(int(vis.sum()) - 0.99 * pos.shape[0]) <= 1
    assert not vis[imp == 0].any()
    assert (vis.astype(bool) == (imp > tau)).all()


def test_visibility_degenerate():
    for mode in (VALUE, MASS):
        vis, tau, _ = oracle.visibility(np.zeros(7), mode=mode)
        assert math.isnan(tau) and not vis.any()
        vis, tau, _ = oracle.visibility(np.array([0.0, 2.0, 0.0]), mode=mode)
        assert tau == 2.0 and not vis.any()             # a single contributor is its own threshold
        vis, _, _ = oracle.visibility(np.zeros(0), mode=mode)
        assert vis.shape == (0,)


def test_critical_identification():
    rng = np.random.default_rng(9)
    n = 5000
    area = rng.integers(0, 4, size=n)
    wmax = rng.random(n)
    crit, tau, _ = oracle.critical(area, wmax, mode=VALUE)
    member = area > 0
    assert tau == pytest.approx(np.quantile(wmax[member], 0.01))
    expect = member & (wmax > tau)
    assert (crit.astype(bool) == expect).all()
    # Gaussians outside G_imax are never critical, whatever their weight
    assert not crit[(area == 0) & (wmax > 0.999)].any()


def test_critical_single_member_is_not_critical():
    for mode in (VALUE, MASS):
        crit, tau, _ = oracle.critical(np.array([0, 3, 0]), np.array([0.9, 0.5, 0.7]), mode=mode)
        assert tau == 0.5 and not crit.any()


def _mass_brute(values, keep):
    """Exact rational prefix sums over the descending order; smallest k on a tie."""
    from fractions import Fraction
    x = sorted((Fraction(v) for v in values), reverse=True)
    S = sum(x)
    best, best_k, C = None, None, Fraction(0)
    for k, v in enumerate(x, 1):
        C += v
        d = abs(C - Fraction(keep) * S)
        if best is None or d < best:
            best, best_k = d, k
    return float(x[best_k - 1])


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("keep", [0.99, 0.9, 0.5, 0.3])
def test_mass_threshold_brute_force(seed, keep):
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(1, 60))
    v = rng.integers(1, 1000, size=m).astype(np.float64) * 2.0 ** -10   # exact in binary
    tau, margin = oracle.threshold(v, keep, MASS)
    if margin > 1e-9:
        assert tau == _mass_brute(v, keep)


def test_mass_threshold_kept_fraction():
    rng = np.random.default_rng(7)
    v = rng.lognormal(sigma=2.0, size=20000)
    tau, _ = oracle.threshold(v, 0.99, MASS)
    kept = v[v > tau].sum() / v.sum()
    gap = tau / v.sum()                                # the element at the threshold, itself not kept
    # C_k* lies within half an element of 0.99 and the kept mass is C_k* - tau
    assert 0.99 - 1.5 * gap <= kept <= 0.99 + 0.5 * gap
    # the heavy tail: far fewer Gaussians than the 99 % kept by count survive
    assert (v > tau).mean() < 0.9


def test_mass_threshold_special_cases():
    assert oracle.threshold(np.array([5.0, 1.0, 1.0]), 1.0, MASS)[0] == 1.0   # C_m = S exactly
    assert oracle.threshold(np.full(100, 0.25), 0.99, MASS)[0] == 0.25     # equal values: nothing above
    assert oracle.threshold(np.array([0.0, 0.0]), 0.99, MASS)[0] == 0.0    # zero total mass
    assert oracle.threshold(np.array([8.0, 1.0]), 0.5, MASS)[0] == 8.0     # C_1 = 8 is nearest to 4.5
    assert oracle.threshold(np.array([4.0, 4.0, 2.0]), 0.6, MASS)[0] == 4.0  # k=2, C=8 nearest 6
    assert math.isnan(oracle.threshold(np.zeros(0), 0.99, MASS)[0])


def test_mass_threshold_tie_prefers_smaller_k():
    # C_1 = 2, C_2 = 4, target 3: equidistant, the smaller k (larger tau) wins
    assert oracle.threshold(np.array([2.0, 2.0, 2.0]), 0.5, MASS)[0] == 2.0
    assert oracle.threshold(np.array([3.0, 2.0, 1.0]), 0.5, MASS)[0] == 3.0   # C = 3 meets target 3


def test_blur_split_threshold_at_paper_constant():
    H, W = 1080, 1920                                   # 2e-4 * H * W = 414.72 pixels
    area = np.array([0, 1, 414, 415, 10**6])
    assert oracle.blur_split(area, H, W).tolist() == [0, 0, 0, 1, 1]
    assert oracle.blur_split(area, H, W, theta=0.0).tolist() == [0, 1, 1, 1, 1]


def _params(n=64, seed=3):
    s = uniform_cube_scene(n, seed=seed)
    return oracle.Params.of(s)


@pytest.mark.parametrize("alpha", [0.01, 0.2, 0.5, 0.9, 0.99])
def test_clone_composite_peak_opacity(alpha):
    p = _params(4)
    p.opacity[:] = alpha
    out = oracle.clone(p, np.array([1, 0, 1, 0]))
    a_new = out.opacity[0]
    assert 1 - (1 - a_new) ** 2 == pytest.approx(alpha, rel=1e-12)
    assert out.opacity[1] == alpha and out.opacity[3] == alpha


@pytest.mark.parametrize("alpha", [0.05, 0.3, 0.7, 0.95])
def test_clone_preserves_line_integral(alpha):
    """Along a line through the centre the screen profile is a 1-D Gaussian whose
    standard deviation scales with the 3-D scales; integrate both opacities."""
    p = _params(1)
    p.opacity[:] = alpha
    out = oracle.clone(p, np.array([1]))
    f = out.scales[0, 0] / p.scales[0, 0]
    a_new = out.opacity[0]
    x = np.linspace(-40.0, 40.0, 400001)
    dx = x[1] - x[0]
    g_old = alpha * np.exp(-0.5 * x * x)
    g_new = a_new * np.exp(-0.5 * (x / f) ** 2)
    comp = 1 - (1 - g_new) ** 2
    assert np.sum(comp) * dx == pytest.approx(np.sum(g_old) * dx, rel=1e-9)


def test_clone_zero_opacity_keeps_scales():
    p = _params(2)
    p.opacity[:] = [0.0, 1.0]
    out = oracle.clone(p, np.array([1, 1]))
    assert out.opacity[0] == 0.0 and (out.scales[:, 0] == p.scales[:, 0]).all()
    assert out.opacity[1] == 1.0
    assert out.scales[0, 1] / p.scales[0, 1] == pytest.approx(1.0 / (2.0 - 2.0 ** -0.5), rel=1e-14)


def test_clone_small_opacity_limit():
    """For small opacity the two copies barely overlap in alpha: a' -> a/2 and the
    scale factor -> 1."""
    p = _params(1)
    p.opacity[:] = 1e-6
    out = oracle.clone(p, np.array([1]))
    assert out.opacity[0] == pytest.approx(0.5e-6, rel=1e-6)
    assert out.scales[0, 0] / p.scales[0, 0] == pytest.approx(1.0, rel=1e-6)


def test_clone_layout_and_copies():
    p = _params(50)
    sel = np.zeros(50, np.uint8)
    sel[[3, 7, 49]] = 1
    out = oracle.clone(p, sel)
    assert out.n == 53
    for j, i in enumerate([3, 7, 49]):
        k = 50 + j
        for a, b in [(out.means, p.means), (out.quats, p.quats)]:
            assert (a[..., k] == b[..., i]).all() and (a[..., i] == b[..., i]).all()
        assert (out.sh[..., k] == p.sh[..., i]).all()
        assert (out.scales[:, k] == out.scales[:, i]).all()
        assert out.opacity[k] == out.opacity[i]
    keep = np.ones(50, bool)
    keep[[3, 7, 49]] = False
    assert (out.scales[:, :50][:, keep] == p.scales[:, keep]).all()
    assert (out.opacity[:50][keep] == p.opacity[keep]).all()
    empty = oracle.clone(p, np.zeros(50, np.uint8))
    assert empty.n == 50 and (empty.scales == p.scales).all()


def test_grad_stats_closed_form():
    """A 3-4-5 gradient in image coordinates; views where the record touches no tile are skipped."""
    V, n = 3, 2
    tiles = np.array([[1, 0], [2, 5], [0, 1]])
    g = np.zeros((V * n, 9))
    W, H = np.array([100, 200, 50]), np.array([80, 60, 40])
    for k in range(V):
        for i in range(n):
            g[k * n + i, 0] = 3.0 / (0.5 * W[k]) * (i + 1)
            g[k * n + i, 1] = -4.0 / (0.5 * H[k]) * (i + 1)
            g[k * n + i, 2:] = 7.0                      # other fields ignored
    ns, cnt = oracle.grad_stats(tiles, g, W, H)
    assert cnt.tolist() == [2, 2]
    assert ns == pytest.approx([2 * 5.0, 2 * 10.0], rel=1e-14)


# --- depth reinitialisation points (Sec. 4.1) and sampling (Sec. 4.2) ---------------

def test_depth_points_round_trip():
    """Lifted points project back onto their pixel centres at their depth."""
    cam = gs_inputs.look_at((1.0, -2.0, 5.0), (0.2, 0.1, 0.0), 40, 30)
    g = np.random.default_rng(3)
    P = cam.width * cam.height
    depth = g.uniform(0.5, 9.0, P)
    imax = np.where(g.uniform(size=P) < 0.8, 7, -1)
    hit = (g.uniform(size=P) < 0.7).astype(np.int32)
    target = g.uniform(size=(3, P))
    u = g.uniform(size=P)
    pts, col = oracle.depth_points(cam, depth, imax, hit, target, u, rate=0.5, require_hit=True)
    keep = np.nonzero((imax >= 0) & (hit > 0) & (u < 0.5))[0]
    assert pts.shape == (keep.size, 3)
    R = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    xc = pts @ R.T + t
    # the float32 rotation is orthonormal to ~1e-7, which bounds the round trip
    np.testing.assert_allclose(xc[:, 2], depth[keep], rtol=1e-6)
    px = xc[:, 0] / xc[:, 2] * cam.fx + cam.cx
    py = xc[:, 1] / xc[:, 2] * cam.fy + cam.cy
    np.testing.assert_allclose(px, keep % cam.width + 0.5, atol=1e-4)
    np.testing.assert_allclose(py, keep // cam.width + 0.5, atol=1e-4)
    np.testing.assert_array_equal(col, target[:, keep].T)
    pts2, _ = oracle.depth_points(cam, depth, imax, hit, target, u, rate=0.5, require_hit=False)
    assert pts2.shape[0] == int(((imax >= 0) & (u < 0.5)).sum())
    assert oracle.depth_points(cam, depth, imax, hit, target, u, rate=0.0)[0].shape == (0, 3)


def _inclusion_exact(w, k):
    """Inclusion probabilities of k sequential draws without replacement, each
    with probability proportional to the remaining weights (enumeration)."""
    import itertools
    n = len(w)
    p = np.zeros(n)
    for seq in itertools.permutations(range(n), k):
        pr, left = 1.0, float(sum(w))
        for i in seq:
            pr *= w[i] / left
            left -= w[i]
        for i in seq:
            p[i] += pr
    return p


@pytest.mark.parametrize("k", [1, 2, 3])
def test_sample_inclusion_probabilities(k):
    w = np.array([1.0, 2.0, 3.0, 0.5, 4.0], np.float32)
    exact = _inclusion_exact([float(x) for x in w], k)
    g = np.random.default_rng(11 + k)
    trials = 20000
    freq = np.zeros(5)
    for _ in range(trials):
        sel = oracle.sample(w, g.exponential(size=5).astype(np.float32), k)
        assert sel.sum() == k
        freq += sel
    freq /= trials
    sd = np.sqrt(exact * (1 - exact) / trials)
    assert (np.abs(freq - exact) <= 4.5 * sd + 1e-12).all(), (freq, exact)


def test_sample_restrictions_and_edges():
    g = np.random.default_rng(5)
    imp = np.array([0.0, 1.0, 2.0, 0.0, 5.0, 1.0], np.float32)
    area = np.array([3, 0, 1, 1, 2, 1], np.uint32)
    e = g.exponential(size=6).astype(np.float32)
    # zero importance is never drawn; area == 0 is outside the intersected set
    assert oracle.sample(imp, e, 10).tolist() == [0, 1, 1, 0, 1, 1]
    assert oracle.sample(imp, e, 10, area).tolist() == [0, 0, 1, 0, 1, 1]
    assert oracle.sample(imp, e, 0).sum() == 0
    # equal weights: the k smallest exponential draws
    eq = np.ones(50, np.float32)
    e = g.exponential(size=50).astype(np.float32)
    sel = oracle.sample(eq, e, 7)
    assert set(np.nonzero(sel)[0]) == set(np.argsort(e, kind="stable")[:7])
    # ties of the key go to the lower index
    assert oracle.sample(np.ones(4, np.float32), np.full(4, 0.5, np.float32), 2).tolist() == [1, 1, 0, 0]
