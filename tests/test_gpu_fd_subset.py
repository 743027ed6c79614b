"""Batched differentiation at full size: 1M Gaussians over 16 views of mixed
resolution in one launch per stage, through the autograd Function with
recompute in backward, L1 loss against a seeded target.  The gradient of one
parameter of each of 256 seeded Gaussians is checked against central finite
differences of the FP64 oracle's loss.  Only the pixels of the perturbed
Gaussian's box change, so the oracle re-renders just those (padded by two
pixels) over the Gaussians whose pixel boxes reach them: every other
Gaussian has alpha below alpha_min there and is skipped by Eq. (1)."""
import numpy as np
import pytest
import torch

import gs_inputs
import oracle
from oracle import F
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu

GROUPS = ("means", "scales", "quats", "opacity", "sh")


def _sub(p, idx):
    return oracle.Params(p.means[:, idx].copy(), p.scales[:, idx].copy(), p.quats[:, idx].copy(),
                         p.opacity[idx].copy(), p.sh[:, :, idx].copy(), p.sh_degree)


def _box_pixels(P, pad):
    xs = np.arange(int(P[F["XLO"]]) - pad, int(P[F["XHI"]]) + pad + 1)
    ys = np.arange(int(P[F["YLO"]]) - pad, int(P[F["YHI"]]) + pad + 1)
    return xs, ys


def test_fd_of_256_gaussians_in_16_view_batch(gpu_lib):
    from paper_2411_12788_amd.autograd import rasterize
    R = H.raster()
    wl = gs_inputs.multiview()
    cams = wl.cameras
    n = wl.scene.n
    lay = R.view_layout(cams)
    Ptot = lay.pixels_total
    target = gs_inputs.uniform_image(3, Ptot, 881)
    ds = R.DeviceScene.from_numpy(wl.scene)
    leaves = [t.clone().requires_grad_(True) for t in (ds.means, ds.scales, ds.quats, ds.opacity, ds.sh)]
    color, _, _ = rasterize(*leaves, cams)
    (color - torch.from_numpy(target).cuda()).abs().mean().backward()
    torch.cuda.synchronize()
    gpu = {k: x.grad.double().cpu().numpy() for k, x in zip(GROUPS, leaves)}
    del leaves, color, ds
    p = oracle.Params.of(wl.scene)
    opts = oracle.Opts()
    projs = [oracle.project(p, c, opts) for c in cams]
    rects = [np.stack([q[:, F["XLO"]], q[:, F["XHI"]], q[:, F["YLO"]], q[:, F["YHI"]]], 1) for q in projs]
    vis = [(q[:, F["VALID"]] == 1) & (q[:, F["TILES"]] > 0) for q in projs]
    nvis = np.sum(vis, axis=0)
    # Gaussians seen in 1..16 views with boxes small enough to re-render quickly
    area = np.max([np.where(vis[v], (r[:, 1] - r[:, 0] + 1) * (r[:, 3] - r[:, 2] + 1), 0)
                   for v, r in enumerate(rects)], axis=0)
    pool = np.nonzero((nvis > 0) & (area <= 400))[0]
    g = gs_inputs.rng(882)
    picks = g.choice(pool, size=256, replace=False)

    class ViewPatch:
        """The Gaussians that can reach the padded box of Gaussian i in view v
        (their pixel boxes overlap it), projected once; the loss over the
        box's pixels is re-evaluated with Gaussian i's parameters replaced."""

        def __init__(self, v, i):
            cam, r = cams[v], rects[v]
            xs, ys = _box_pixels(projs[v][i], 2)
            x0, x1, y0, y1 = xs[0], xs[-1], ys[0], ys[-1]
            near = np.nonzero(vis[v] & (r[:, 1] >= x0) & (r[:, 0] <= x1) & (r[:, 3] >= y0) & (r[:, 2] <= y1))[0]
            self.near = np.union1d(near, [i])
            self.j = int(np.searchsorted(self.near, i))
            self.sub = _sub(p, self.near)
            self.qs = oracle.project(self.sub, cam, opts)
            X, Y = np.meshgrid(np.clip(xs, 0, cam.width - 1), np.clip(ys, 0, cam.height - 1))
            self.pix = np.unique(np.stack([X.ravel(), Y.ravel()], 1), axis=0).astype(np.int32)
            gi = lay.pixel_base[v] + self.pix[:, 1] * cam.width + self.pix[:, 0]
            self.t = target[:, gi].T
            self.cam = cam

        def loss(self, pp_i):
            sub = self.sub.copy()
            for k in GROUPS:
                getattr(sub, k)[..., self.j] = getattr(pp_i, k)[..., 0]
            qs = self.qs.copy()
            qs[self.j] = oracle.project(pp_i, self.cam, opts)[0]
            out = oracle.render(sub, self.cam, qs, oracle.order(qs), opts, pixels=self.pix, accumulate=False)
            return float(np.abs(out["color"] - self.t).sum())

    fd, gp, skipped = [], [], 0
    for i in picks:
        k = GROUPS[int(g.integers(0, len(GROUPS)))]
        shape = getattr(p, k).shape[:-1]
        comp = tuple(int(g.integers(0, s)) for s in shape)
        if k == "sh":
            comp = (int(g.integers(0, 16)), int(g.integers(0, 3)))
        x = float(getattr(p, k)[comp + (i,)])
        vals = []
        patches = [ViewPatch(v, i) for v in range(len(cams)) if vis[v][i]]
        for h in (1e-7 * max(1.0, abs(x)), 0.5e-7 * max(1.0, abs(x))):
            tot = 0.0
            for sgn in (1.0, -1.0):
                pp = _sub(p, [i])
                getattr(pp, k)[comp + (0,)] = x + sgn * h
                tot += sgn * sum(pt.loss(pp) for pt in patches)
            vals.append(tot / (2 * h) / (3.0 * Ptot))
        # a decision (skip / stop / clamp / |.| kink) inside the step makes the
        # difference quotient depend on h: such samples are not smooth there
        if abs(vals[0] - vals[1]) > 1e-3 * max(abs(vals[0]), 1e-12):
            skipped += 1
            continue
        fd.append(vals[1])
        gp.append(gpu[k][comp + (i,)])
    fd, gp = np.array(fd), np.array(gp)
    H.report("fd subset 1M x 16 views", samples=len(fd), skipped=skipped, rel_l2=H.rel_l2(gp, fd))
    assert len(fd) >= 200, (len(fd), skipped)
    assert H.rel_l2(gp, fd) <= H.GRAD_REL_L2
