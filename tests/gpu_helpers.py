"""Shared helpers for GPU parity tests: run the HIP path and the oracle on the
same seeded inputs and compare with the stated tolerances."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from oracle import F

# Tolerances.
COLOR_ATOL = 1e-4        # colour and depth, max abs over non-ambiguous pixels
GRAD_REL_L2 = 1e-3       # per parameter group
# A pixel is ambiguous when float32 and float64 may legitimately take a
# different discrete decision there: an evaluated alpha within 2e-5 (relative)
# of the skip threshold, a transmittance within 2e-3 (relative; (1 - alpha)
# amplifies alpha's error up to 100x at alpha = 0.99) of the stop threshold.
# For the argmax index (and depth), also when the top-two weights are within 1e-4.
ALPHA_MARGIN = 2e-5
STOP_MARGIN = 2e-3
ARGMAX_MARGIN = 1e-4
MAX_AMBIGUOUS_FRACTION = 3e-3


def raster():
    from paper_2411_12788_amd import raster as R
    return R


def oracle_opts(opts=None, **kw):
    o = oracle.Opts(**kw)
    return o


def gpu_opts(**kw):
    R = raster()
    return R.RasterOpts(**kw)


def run_gpu_forward(scene, cams, opts=None, cull=None, accumulate=True, per_view=False, want_keys=False):
    R = raster()
    opts = opts or R.RasterOpts()
    ds = R.DeviceScene.from_numpy(scene)
    cm = None if cull is None else torch.from_numpy(cull).cuda()
    proj = R.project(ds, cams, opts, cm)
    binned = R.bin(proj, cams, ds.n, want_keys=want_keys)
    acc = R.alloc_accum(ds.n, len(cams), per_view) if accumulate else None
    if accumulate and per_view:
        opts = R.RasterOpts(**{**opts.__dict__, "flags": opts.flags | 2})
    frame = R.render_forward(ds, proj, binned, cams, opts, accum=acc)
    torch.cuda.synchronize()
    return dict(scene=ds, proj=proj, binned=binned, frame=frame, acc=acc, opts=opts)


def ambiguous(orc_out, argmax=False):
    m = orc_out["margin"]
    amb = (m[:, 0] < ALPHA_MARGIN) | (m[:, 1] < STOP_MARGIN)
    if argmax:
        amb |= m[:, 2] < ARGMAX_MARGIN
    return amb


def view_slice(layout, v):
    lo = layout.pixel_base[v]
    return slice(lo, lo + (layout.pixel_base[v + 1] if v + 1 < len(layout.pixel_base) else layout.pixels_total) - lo)


def compare_forward(gpu_frame, orc, pix_slice, what="", max_ambiguous=MAX_AMBIGUOUS_FRACTION):
    """Checks one view's GPU outputs against the oracle's full-image outputs;
    at most a fraction max_ambiguous of the pixels may be ambiguous."""
    col = gpu_frame.color[:, pix_slice].T.double().cpu().numpy()
    amb = ambiguous(orc)
    amb_arg = ambiguous(orc, argmax=True)
    # binomial headroom for small images: a handful of pixels on top of the rate
    assert amb_arg.sum() <= max_ambiguous * amb_arg.size + 10, (what, int(amb_arg.sum()), amb_arg.size)
    ok = ~amb
    err = np.abs(col - orc["color"])[ok]
    assert err.size == 0 or err.max() <= COLOR_ATOL, (what, err.max())
    tf = gpu_frame.t_final[pix_slice].double().cpu().numpy()
    assert np.abs(tf - orc["t_final"])[ok].max(initial=0) <= COLOR_ATOL, what
    nc = gpu_frame.n_contrib[pix_slice].cpu().numpy()
    assert np.array_equal(nc[ok], orc["n_contrib"][ok]), what
    ok2 = ~amb_arg
    im = gpu_frame.imax[pix_slice].cpu().numpy()
    assert np.array_equal(im[ok2], orc["imax"][ok2]), what
    dep = gpu_frame.depth[pix_slice].double().cpu().numpy()
    derr = np.abs(dep - orc["depth"])[ok2]
    assert derr.size == 0 or derr.max() <= COLOR_ATOL, (what, derr.max())
    hit = gpu_frame.hit[pix_slice].cpu().numpy()
    mism = (hit[ok2] != orc["hit"][ok2]).sum()
    assert mism <= 2 + 1e-4 * ok2.sum(), (what, mism)
    return amb, amb_arg


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
