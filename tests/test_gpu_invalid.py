"""Invalid Gaussians mixed into a valid scene, through the GPU path: a zero
quaternion, non-finite means, scales and opacities, opacity below alpha_min,
centres behind the near plane or the camera, and colours that
are not finite.  Each is excluded at projection (Sec. 3.1; tiles_touched = 0 and no
key), exactly as in the oracle, the image equals the oracle's over the valid
Gaussians, and the backward writes finite gradients with zero rows for the
excluded ones."""
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


def _scene_with_invalid(n=1500, seed=21):
    sc = gs_inputs.uniform_cube_scene(n, seed)
    bad = {}
    k = 0

    def take(tag):
        nonlocal k
        bad[tag] = k * 37 + 5  # spread over the index range
        k += 1
        return bad[tag]

    sc.quats[:, take("zero quaternion")] = 0.0
    sc.means[0, take("nan mean")] = np.nan
    sc.means[2, take("inf mean")] = np.inf
    sc.scales[1, take("nan scale")] = np.nan
    sc.opacity[take("opacity below alpha_min")] = np.float32(0.5 / 255.0)
    sc.opacity[take("zero opacity")] = 0.0
    sc.opacity[take("nan opacity")] = np.nan
    i = take("behind near plane")
    sc.means[:, i] = (0.0, 0.0, 3.9)  # camera at z = 4 looking at the origin: depth 0.1 < znear
    i = take("behind camera")
    sc.means[:, i] = (0.0, 0.0, 6.0)
    sc.sh[0, :, take("inf colour")] = np.inf
    sc.sh[5, 1, take("nan sh")] = np.nan
    return sc, bad


def test_invalid_gaussians_are_excluded(gpu_lib):
    R = H.raster()
    sc, bad = _scene_with_invalid()
    cam = gs_inputs.look_at((0, 0, 4), (0, 0, 0), 96, 72)
    n, Pn = sc.n, cam.width * cam.height
    out = H.run_gpu_forward(sc, [cam], accumulate=True, want_keys=True)
    binr = _np(out["proj"].bin)
    p = oracle.Params.of(sc)
    orc = oracle.forward_view(p, cam, oracle.Opts())
    P = orc["proj"]
    for tag, i in bad.items():
        assert P[i, F["VALID"]] == 0, tag
        assert binr[i, 3] == 0, tag
    vis_o = (P[:, F["VALID"]] == 1) & (P[:, F["TILES"]] > 0)
    assert np.array_equal(vis_o, binr[:, 3] > 0)
    assert vis_o.sum() > n // 2
    # no key of an excluded Gaussian
    vals = _np(out["binned"].vals).view(np.uint32)
    assert not np.isin(vals, np.array(list(bad.values()), dtype=np.uint32)).any()
    # the image and the sums equal the oracle's over the valid Gaussians
    flips, _ = H.compare_forward(out["frame"], orc, slice(0, Pn), "invalid inputs", p, cam)
    H.check_accum(out["acc"], p, cam, P, orc["order"], oracle.Opts(), flips, n, "invalid inputs")
    acc = {k: _np(v) for k, v in out["acc"].items()}
    for i in bad.values():
        assert acc["importance"][i] == 0 and acc["wmax"][i] == 0 and acc["area"][i] == 0
    # backward: finite everywhere, zero on excluded rows, oracle parity elsewhere
    dldc = gs_inputs.normal_image(3, Pn, 23, scale=1.0 / Pn)
    grads, g2d = R.render_backward(out["scene"], out["proj"], out["binned"], [cam], R.RasterOpts(), out["frame"],
                                   torch.from_numpy(dldc).cuda())
    torch.cuda.synchronize()
    og, _ = H.backward_views(p, [cam], oracle.Opts(), [dldc.T.astype(np.float64)], flips=[flips])
    g2 = _np(g2d)
    assert np.isfinite(g2).all()
    idx = np.array(list(bad.values()))
    assert np.all(g2[idx] == 0)
    for k in ("means", "scales", "quats", "opacity", "sh"):
        gk = _np(grads[k]).astype(np.float64)[..., :n]
        assert np.isfinite(gk).all(), k
        assert np.all(gk[..., idx] == 0), k
        assert H.rel_l2(gk, og[k]) <= H.GRAD_REL_L2, k
