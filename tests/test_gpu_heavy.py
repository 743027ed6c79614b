"""Parity on heavy tiles: every tile's list holds thousands of entries, so the
renderer takes its split path (a long tile is shared by four workgroups, one
4x4 pixel group per wave).  Faint Gaussians make pixels composite hundreds of
entries (Eq. (1)); brighter ones make them reach the transmittance stop
inside long streams.  Forward outputs and accumulations against the oracle's
per-pixel definition, gradients by relative L2, both with the active mask."""
import numpy as np
import pytest
import torch

import gs_inputs
import oracle
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("opacity", [(0.01, 0.05), (0.05, 0.3)])
def test_heavy_tiles_forward_backward(gpu_lib, opacity):
    R = H.raster()
    wl = gs_inputs.heavy_tiles(seed=7, opacity=opacity)
    cam = wl.cameras[0]
    n, Pn = wl.scene.n, cam.width * cam.height
    out = H.run_gpu_forward(wl.scene, wl.cameras, accumulate=True)
    rng = _np(out["binned"].ranges).reshape(-1, 2)
    assert ((rng[:, 1] - rng[:, 0]) >= 2048).all()  # every tile is a heavy one
    p = oracle.Params.of(wl.scene)
    orc = oracle.forward_view(p, cam, oracle.Opts())
    # most bright pixels stop inside their stream, and many stops are decided
    # within the float32 error of the threshold: those pixels are checked
    # against both branches
    flips, namb = H.compare_forward(out["frame"], orc, slice(0, Pn), f"heavy tiles {opacity}", p, cam)
    H.check_accum(out["acc"], p, cam, orc["proj"], orc["order"], oracle.Opts(), flips, n, f"heavy tiles {opacity}")
    if opacity[1] > 0.1:
        assert (orc["t_final"] < 1e-3).mean() > 0.2  # the stop is reached inside the streams
    dldc = gs_inputs.normal_image(3, Pn, 31, scale=1.0 / Pn)
    active = gs_inputs.bernoulli_mask(n, 0.25, 32)
    grads, g2d = R.render_backward(out["scene"], out["proj"], out["binned"], wl.cameras, R.RasterOpts(),
                                   out["frame"], torch.from_numpy(dldc).cuda(), torch.from_numpy(active).cuda())
    torch.cuda.synchronize()
    og, og2d = H.backward_views(p, wl.cameras, oracle.Opts(), [dldc.T.astype(np.float64)], active=active,
                                flips=[flips])
    g2 = _np(g2d).astype(np.float64)[:n]
    assert H.rel_l2(g2, og2d[0] * active[:, None]) <= H.GRAD_REL_L2
    for k in ("means", "scales", "quats", "opacity", "sh"):
        gk = _np(grads[k])[..., :n].astype(np.float64)
        assert H.rel_l2(gk, og[k]) <= H.GRAD_REL_L2, k


def test_concentrated_heavy_tiles_forward_backward(gpu_lib):
    """Most tiles empty, a few with long lists: the forward takes its
    row-parallel split form (the four rows of a wave are consecutive entries
    of one pixel group's stream) as well as the backward."""
    R = H.raster()
    wl = gs_inputs.heavy_tiles(seed=9, n=20_000, width=128, height=96, opacity=(0.02, 0.2), distance=9.0)
    cam = wl.cameras[0]
    n, Pn = wl.scene.n, cam.width * cam.height
    out = H.run_gpu_forward(wl.scene, wl.cameras, accumulate=True)
    rng = _np(out["binned"].ranges).reshape(-1, 2)
    lens = rng[:, 1] - rng[:, 0]
    assert (lens == 0).mean() > 0.5 and (lens >= 256).sum() >= 4
    p = oracle.Params.of(wl.scene)
    orc = oracle.forward_view(p, cam, oracle.Opts())
    assert (orc["t_final"] < 1e-3).sum() > 100  # pixels that stop inside the four-entry steps
    flips, _ = H.compare_forward(out["frame"], orc, slice(0, Pn), "concentrated heavy tiles", p, cam)
    H.check_accum(out["acc"], p, cam, orc["proj"], orc["order"], oracle.Opts(), flips, n, "concentrated heavy tiles")
    dldc = gs_inputs.normal_image(3, Pn, 41, scale=1.0 / Pn)
    active = gs_inputs.bernoulli_mask(n, 0.25, 42)
    grads, g2d = R.render_backward(out["scene"], out["proj"], out["binned"], wl.cameras, R.RasterOpts(),
                                   out["frame"], torch.from_numpy(dldc).cuda(), torch.from_numpy(active).cuda())
    torch.cuda.synchronize()
    og, og2d = H.backward_views(p, wl.cameras, oracle.Opts(), [dldc.T.astype(np.float64)], active=active,
                                flips=[flips])
    assert H.rel_l2(_np(g2d).astype(np.float64)[:n], og2d[0] * active[:, None]) <= H.GRAD_REL_L2
    for k in ("means", "scales", "quats", "opacity", "sh"):
        assert H.rel_l2(_np(grads[k])[..., :n].astype(np.float64), og[k]) <= H.GRAD_REL_L2, k

