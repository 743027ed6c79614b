#!/usr/bin/env python3
"""Benchmark: one training step of the rasterizer hot path on one MI355X.

A step is one pass of the whole path over one synthetic view: projection (a1),
binning count + key emission + sort + tile ranges (a2-a4), forward compositing
with fused importance / max-weight / area accumulation (a5-a6), the L1 loss
gradient, the masked reverse-order backward (a7) and the projection backward
(a8).  Default workload: 3M surface-sampled Gaussians, one 1920x1080 view,
25% of Gaussians active in the backward.

Prints one JSON line (metric, value = ms/step, roofline of the dominant kernel
measured with HIP events on the launch stream, CPU-oracle baseline).
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import gs_inputs  # noqa: E402

PEAK_HBM_GBS = 8000.0
# FP32 VALU issue rate without packed FP32 (disabled in this build): 256 CUs x
# 4 SIMDs x 16 lanes per clock x 2.4 GHz = 39.3 T lane-ops/s
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
STOP_T = 0.01  # a pixel with final transmittance >= 1e-4 / (1 - 0.99) never stopped
# algorithmic bytes per unit: what each kernel must read and write at least
PROJECT_BYTES_PER_RECORD = 59 * 4 + 64 + 16     # drawn: params read, record + bin written
PROJECT_BYTES_PER_UNDRAWN = 11 * 4 + 16          # not drawn: no SH read (mean, scale, rotation, opacity), no record
PROJECT_BWD_BYTES_PER_ACTIVE = 59 * 4 + 59 * 4 + 36 + 16  # params read, grads written, 2D grad + bin read
PROJECT_BWD_BYTES_PER_INACTIVE = 59 * 4 + 1     # zero rows written, mask read
RENDER_FWD_BYTES_PER_PAIR = 4 + 8 + 48          # list index, pixel box, the 48 record bytes compositing reads
RENDER_FWD_BYTES_PER_PIXEL = 12 + 4 + 4 + 4 + 4 + 4 + 1  # colour, depth, imax, T, last, count, hit
RENDER_BWD_BYTES_PER_PAIR = 4 + 8 + 64 + 1      # list index, box, full record, active flag
RENDER_BWD_BYTES_PER_PIXEL = 12 + 4 + 4         # dL/dC, T, last
BIN_PARTS = {"count": ["k_count_reduce", "k_count_down"],
             "sort": ["k_emit", "k_rt_up", "k_rt_scan", "k_os_hist", "k_os_scan", "k_os_pass", "k_ranges",
                      "k_tile_order", "k_order_hist", "k_order_scan", "k_order_scatter"]}
STAGE_KERNELS = {"project": ["k_project"], "bin": BIN_PARTS["count"] + BIN_PARTS["sort"],
                 "render_fwd": ["k_render_fwd"], "loss": ["k_l1_loss_grad"], "render_bwd": ["k_render_bwd"],
                 "project_bwd": ["k_project_bwd1", "k_project_bwd"]}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large", choices=["large", "training", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cores", type=int, default=0, help="oracle baseline processes (default: host cores, <= 16)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-warmup", type=int, default=200)
    ap.add_argument("--no-multiview", action="store_true")
    ap.add_argument("--no-criteria", action="store_true")
    ap.add_argument("--input-order", action="store_true",
                    help="time the Gaussians in their generated order instead of the library's spatial order")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: a few steps plus a 1 GiB copy kernel for counter calibration")
    ap.add_argument("--summarize", metavar="DIR",
                    help="write profiles/ summaries from rocprofv3 output in DIR (kt/, fetch/, write/ sub-folders)")
    return ap.parse_args()


def workload(name):
    if name == "large":
        return gs_inputs.large_scene()
    if name == "training":
        wl = gs_inputs.training_view()
        wl.active = gs_inputs.bernoulli_mask(wl.scene.n, 0.25, 2001)
        return wl
    wl = gs_inputs.small_cube()
    wl.active = gs_inputs.bernoulli_mask(wl.scene.n, 0.25, 2002)
    return wl


class Step:
    """Buffers and launches of one training step (all on torch's current stream)."""

    def __init__(self, wl, spatial: bool = True):
        from paper_2411_12788_amd import raster as R
        self.R = R
        self.cams = wl.cameras
        self.opts = R.RasterOpts()
        self.scene = R.DeviceScene.from_numpy(wl.scene)
        self.n = self.scene.n
        self.lay = R.view_layout(self.cams)
        P = self.lay.pixels_total
        self.target = torch.from_numpy(gs_inputs.uniform_image(3, P, 4242)).cuda()
        self.active = torch.from_numpy(wl.active).cuda() if wl.active is not None else None
        self.perm = None
        if spatial:
            # the layout the library keeps Gaussians in: the same set, stored
            # along the Morton curve of the means; the mask moves with them
            self.scene, self.perm = self.scene.in_spatial_order()
            if self.active is not None:
                self.active = R.permute(self.active, self.perm)
        self.dldc = torch.empty((3, P), device="cuda")
        # what the step clears (accumulators, loss, the per-record 2D gradient
        # the backward adds into) lives in one arena: one fill clears it
        n, V = self.n, len(self.cams)
        pieces = {"importance": n, "wmax": n, "area": n, "loss": 1, "grad2d": 9 * n * V}
        at, offs = 0, {}
        for k, c in pieces.items():
            offs[k] = at
            at += (c + 63) // 64 * 64  # 256-byte aligned pieces
        self.arena = torch.zeros(at, device="cuda")
        cut = {k: self.arena[offs[k]: offs[k] + c] for k, c in pieces.items()}
        self.acc = dict(importance=cut["importance"], wmax=cut["wmax"], area=cut["area"].view(torch.int32))
        self.loss = cut["loss"]
        self.grad2d = cut["grad2d"].view(n * V, 9)
        self.grads = R.alloc_grads(self.n)
        self.names = ["project", "bin", "render_fwd", "loss", "render_bwd", "project_bwd"]
        self.pending = []  # recorded steps whose events are read after the timed region
        self.prepared = []  # event sets made ahead of the timed region
        self.times = {k: [] for k in self.names}
        self.frame = None
        self.buffers = R.StepBuffers()  # pair count, lists and sort workspace, reused

    def run(self, record: bool, recompute: bool = False):
        """One step.  With `recompute` the backward re-derives the projection
        and the sorted lists instead of keeping the forward's (the memory-lean
        mode of the autograd wrapper)."""
        R = self.R
        if record:
            # one set of events per step, read once after the timed region (no
            # synchronisation between steps), created beforehand by
            # prepare_events (creating them here made a rare host stall of
            # ~1 ms inside the timed region)
            ev = self.prepared.pop() if self.prepared else self._new_events()
            self.pending.append(ev)

        def mark(k, i):
            if record:
                ev[k][i].record()

        # The clears the step needs (accumulators, loss, the per-record 2D
        # gradient the backward adds into), one fill over their arena, queued
        # first: the device is still busy with the previous step's backward,
        # so the launch costs no idle time.  Queued after the pair count
        # instead, it would be a gap: nothing else is queued then.
        R.fill_u32(self.arena, 0)
        mark("project", 0)
        proj = R.project(self.scene, self.cams, self.opts, buffers=self.buffers)
        mark("project", 1)
        mark("bin", 0)
        binned = R.bin_step(proj, self.cams, self.n, self.buffers)
        mark("bin", 1)
        mark("render_fwd", 0)
        self.frame = R.render_forward(self.scene, proj, binned, self.cams, self.opts, accum=self.acc,
                                      extras=True, out=self.frame)
        mark("render_fwd", 1)
        mark("loss", 0)
        R.l1_loss_grad(self.frame.color, self.target, self.dldc, self.loss)
        mark("loss", 1)
        if recompute:
            proj = R.project(self.scene, self.cams, self.opts, buffers=self.buffers)
            binned = R.bin_step(proj, self.cams, self.n, self.buffers)
        mark("render_bwd", 0)
        R.render_backward_pixels(proj, binned, self.cams, self.n, self.opts, self.frame, self.dldc, self.active,
                                 self.grad2d)
        mark("render_bwd", 1)
        mark("project_bwd", 0)
        from paper_2411_12788_amd import _lib as L
        import ctypes
        L.check(L.lib().gs_project_backward(ctypes.byref(self.scene.c()), ctypes.byref(proj.c()),
                                            R.cameras(self.cams), len(self.cams), ctypes.byref(self.opts.c()),
                                            ctypes.c_void_p(self.grad2d.data_ptr()),
                                            None if self.active is None else ctypes.c_void_p(self.active.data_ptr()),
                                            ctypes.byref(R._grads_c(self.grads)), R._stream()), "project_backward")
        mark("project_bwd", 1)
        self.stats = binned.stats
        self.proj = proj
        self.binned = binned

    def _new_events(self):
        return {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in self.names}

    def prepare_events(self, steps: int):
        """Create (and record once, so the device events exist) the event sets
        of `steps` recorded steps."""
        self.prepared = [self._new_events() for _ in range(steps)]
        for ev in self.prepared:
            for a, b in ev.values():
                a.record()
                b.record()
        torch.cuda.synchronize()

    def collect(self):
        """Stage times of the recorded steps (after a synchronisation)."""
        torch.cuda.synchronize()
        for ev in self.pending:
            for k in self.names:
                self.times[k].append(ev[k][0].elapsed_time(ev[k][1]))
        self.pending = []


def spatial_order_ms(step, reps: int = 5) -> float:
    """One-off cost of moving the step's scene (generated order) and mask into
    the spatial order: Morton codes, their sort, and the planar gathers."""
    R = step.R

    def one():
        sc, perm = step.scene.in_spatial_order()
        if step.active is not None:
            R.permute(step.active, perm)
        return sc

    one()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        one()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def pair_evaluations(step):
    """(forward, backward) pair-evaluations of the tile algorithm for the last
    step of a one-view workload: per pixel the length of its tile's list, or
    for a pixel that may have stopped (T_final < STOP_T) its last contributor
    (a lower bound of where it stopped); backward: the last contributor."""
    assert len(step.cams) == 1
    cam = step.cams[0]
    W, H = cam.width, cam.height
    tx = (W + 15) // 16
    rng = step.binned.ranges.view(-1, 2).long()
    L = rng[:, 1] - rng[:, 0]
    py = torch.arange(H, device="cuda").view(H, 1) // 16
    px = torch.arange(W, device="cuda").view(1, W) // 16
    Lp = L[(py * tx + px).reshape(-1)]
    P = W * H
    last = step.frame.last[:P].long()
    tf = step.frame.t_final[:P]
    fwd = torch.where(tf >= STOP_T, Lp, last).sum().item()
    return float(fwd), float(last.sum().item())


def deterministic_backward_ms(step, reps: int = 10) -> float:
    """Time of the pixel backward of the last timed step with the ordered,
    atomic-free reduction (bitwise-reproducible gradients), workspace reused."""
    from paper_2411_12788_amd import _lib as L
    R = step.R
    ni = int(step.binned.stats.n_isect)
    ws = torch.empty(max(L.lib().gs_render_backward_det_workspace_size(ni), 1), dtype=torch.uint8, device="cuda")

    def one():
        step.grad2d.zero_()
        R.render_backward_pixels(step.proj, step.binned, step.cams, step.n, step.opts, step.frame, step.dldc,
                                 step.active, step.grad2d, deterministic=True, det_ws=ws)

    one()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    total = 0.0
    for _ in range(reps):
        step.grad2d.zero_()
        e0.record()
        R.render_backward_pixels(step.proj, step.binned, step.cams, step.n, step.opts, step.frame, step.dldc,
                                 step.active, step.grad2d, deterministic=True, det_ws=ws)
        e1.record()
        torch.cuda.synchronize()
        total += e0.elapsed_time(e1)
    return total / reps


def bin_sort_ms(step, algorithm: int, reps: int = 10) -> float:
    """Time of the bin_sort stage of the last timed step with the given radix
    pass algorithm (GS_SORT_PRESCAN or GS_SORT_LOOKBACK), same buffers."""
    from paper_2411_12788_amd import _lib as L
    R = step.R
    L.check(L.lib().gs_sort_set_algorithm(algorithm), "gs_sort_set_algorithm")
    try:
        offsets, st = R.bin_count(step.proj, step.cams, step.n)
        R.bin_sort(step.proj, step.cams, step.n, offsets, st, buffers=step.buffers.bins)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        total = 0.0
        for _ in range(reps):
            e0.record()
            R.bin_sort(step.proj, step.cams, step.n, offsets, st, buffers=step.buffers.bins)
            e1.record()
            torch.cuda.synchronize()
            total += e0.elapsed_time(e1)
        R.sort_status(step.buffers.bins.ws)
    finally:
        L.lib().gs_sort_set_algorithm(L.GS_SORT_PRESCAN)
    return total / reps


def criteria_bench(step, reps: int = 10):
    """Time the culling/densification criteria on the accumulations of the last
    timed step: per-view visibility and critical set (both threshold readings),
    blur split, two-way clone of the critical set, gradient statistics, the
    3DGS clone/split selection and the split of the critical set.
    'gbs' uses the algorithmic minimum traffic (read the inputs once, write the
    outputs once), so it is a lower bound on what the kernels move."""
    from paper_2411_12788_amd import densify as Dz
    n = step.n
    imp = step.acc["importance"].view(1, n)
    area, wmax = step.acc["area"], step.acc["wmax"]
    from paper_2411_12788_amd import _lib as L
    ws = torch.empty(L.lib().gs_select_workspace_size(1), dtype=torch.uint8, device="cuda")
    res = {}

    def timed(name, fn, nbytes):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            out = fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"ms": round(ms, 4), "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1)}
        return out

    for mode, tag in ((Dz.THRESHOLD_MASS, "mass"), (Dz.THRESHOLD_VALUE, "value")):
        timed(f"visibility_{tag}", lambda: Dz.visibility(imp, mode=mode, ws=ws), 5 * n)
        crit = timed(f"critical_{tag}", lambda: Dz.critical(area, wmax, mode=mode, ws=ws), 9 * n)
    sel = crit[0]
    cnt = int(sel.sum().item())
    res["critical_count"] = cnt
    timed("blur_split", lambda: Dz.blur_split(area, step.cams[0].height, step.cams[0].width), 5 * n)
    timed("clone", lambda: Dz.clone(step.scene, sel, capacity=n + cnt), 236 * n + 1 * n + 236 * (n + cnt))
    ns = torch.zeros(n, device="cuda")
    cn = torch.zeros(n, dtype=torch.int32, device="cuda")
    timed("grad_stats", lambda: Dz.grad_stats(step.proj, step.grad2d, step.cams, n, ns, cn), 28 * n)
    timed("densify_select", lambda: Dz.densify_select(ns, cn, step.scene.scales, 2e-4, 0.05), 22 * n)
    z = torch.randn((2, 3, n), generator=torch.Generator(device="cuda").manual_seed(7), device="cuda")
    timed("split", lambda: Dz.split(step.scene, sel, z, capacity=n + cnt), 236 * n + n + 24 * cnt + 236 * (n + cnt))
    return res


# --------------------------------------------------------------------------
# CPU baseline: the FP64 oracle over the host's cores
# --------------------------------------------------------------------------
_CPU = {}  # read by the forked workers (copy-on-write)


def _cpu_project(sl):
    import oracle
    c = _CPU
    p = c["params"]
    sub = oracle.Params(p.means[:, sl], p.scales[:, sl], p.quats[:, sl], p.opacity[sl], p.sh[:, :, sl], p.sh_degree)
    t = time.process_time()
    out = oracle.project(sub, c["cam"], c["opts"])
    return sl, out, time.process_time() - t


def _band_pixels(ty):
    cam = _CPU["cam"]
    y0, y1 = 16 * ty, min(16 * ty + 16, cam.height)
    ys, xs = np.mgrid[y0:y1, 0:cam.width]
    return np.stack([xs.ravel(), ys.ravel()], 1).astype(np.int32)


def _cpu_render(ty):
    import oracle
    c = _CPU
    pix = _band_pixels(ty)
    t = time.process_time()
    r = oracle.render(c["params"], c["cam"], c["proj"], c["order"], c["opts"], pixels=pix, tiles=c["tiles"],
                      accumulate=True)
    cpu = time.process_time() - t
    nz = np.nonzero(r["importance"])[0]
    acc = (nz, r["importance"][nz], r["wmax"][nz], r["area"][nz])
    return ty, r["color"], r["t_final"], r["imax"], acc, cpu


def _cpu_backward(ty):
    import oracle
    c = _CPU
    pix = _band_pixels(ty)
    idx = pix[:, 1] * c["cam"].width + pix[:, 0]
    t = time.process_time()
    g2d = oracle.render_backward(c["params"], c["cam"], c["proj"], c["order"], c["opts"], c["dldc"][idx],
                                 pixels=pix, tiles=c["tiles"])
    cpu = time.process_time() - t
    nz = np.nonzero(np.any(g2d != 0, axis=1))[0]
    return nz, g2d[nz], cpu


def _cpu_project_backward(sl):
    import oracle
    c = _CPU
    p = c["params"]
    sub = oracle.Params(p.means[:, sl], p.scales[:, sl], p.quats[:, sl], p.opacity[sl], p.sh[:, :, sl], p.sh_degree)
    t = time.process_time()
    g = oracle.project_backward(sub, c["cam"], c["opts"], c["proj"][sl], c["g2d"][sl])
    return sl, g, time.process_time() - t


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, cores: int = 0):
    """The FP64 oracle as it stands, timed on the host's cores over the whole
    step of the same workload: projection, depth order and binning, the
    tile-restricted forward with the three accumulations over every pixel, the
    L1 loss gradient, the backward over every pixel, and the projection
    backward with the active mask.  Per-Gaussian stages are split over chunks
    of Gaussians and per-pixel stages over 16-pixel rows of tiles, across a
    pool of forked processes (one per core, at most 16).  Stage times are wall
    clock; the summed process CPU time gives the one-core figure."""
    import multiprocessing as mp
    import oracle
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = cores or min(16, avail)
    cam = wl.cameras[0]
    n, W, H = wl.scene.n, cam.width, cam.height
    P = W * H
    _CPU.clear()
    _CPU.update(params=oracle.Params.of(wl.scene), cam=cam, opts=oracle.Opts())
    target = gs_inputs.uniform_image(3, P, 4242).T.astype(np.float64)
    chunks = [slice(a, min(a + 65536, n)) for a in range(0, n, 65536)]
    bands = list(range((H + 15) // 16))
    times, cpu = {}, 0.0
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    proj = np.zeros((n, oracle.STRIDE))
    with ctx.Pool(cores) as pool:
        for sl, out, c in pool.imap_unordered(_cpu_project, chunks):
            proj[sl] = out
            cpu += c
    times["project"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    c0 = time.process_time()
    ordr = oracle.order(proj)
    tx, ty, base, total = oracle.view_layout([cam])
    _, vals, ranges = oracle.bin(oracle.tile_rects(proj), oracle.zbits(proj), 1, n, base, tx, total)
    cpu += time.process_time() - c0
    times["order_and_bin"] = time.perf_counter() - t0
    _CPU.update(proj=proj, order=ordr, tiles=(vals, ranges))
    t0 = time.perf_counter()
    color = np.zeros((P, 3))
    imp, wmax, area = np.zeros(n), np.zeros(n), np.zeros(n, dtype=np.int64)
    with ctx.Pool(cores) as pool:
        for tyk, col, tf, im, (nz, a_i, a_w, a_s), c in pool.imap_unordered(_cpu_render, bands):
            y0 = 16 * tyk
            color[y0 * W:y0 * W + col.shape[0]] = col
            imp[nz] += a_i
            np.maximum.at(wmax, nz, a_w)
            area[nz] += a_s
            cpu += c
    times["render_forward"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    c0 = time.process_time()
    dldc = np.sign(color - target) / (3.0 * P)
    cpu += time.process_time() - c0
    times["loss"] = time.perf_counter() - t0
    _CPU.update(dldc=dldc)
    t0 = time.perf_counter()
    g2d = np.zeros((n, 9))
    with ctx.Pool(cores) as pool:
        for nz, rows, c in pool.imap_unordered(_cpu_backward, bands):
            g2d[nz] += rows
            cpu += c
    times["render_backward"] = time.perf_counter() - t0
    _CPU.update(g2d=g2d)
    t0 = time.perf_counter()
    grads = {}
    with ctx.Pool(cores) as pool:
        for sl, g, c in pool.imap_unordered(_cpu_project_backward, chunks):
            for k, v in g.items():
                grads.setdefault(k, np.zeros(v.shape[:-1] + (n,)))[..., sl] = v
            cpu += c
    if wl.active is not None:
        for v in grads.values():
            v[..., wl.active == 0] = 0.0
    times["project_backward"] = time.perf_counter() - t0
    _CPU.clear()
    ms = 1e3 * sum(times.values())
    return {"value": round(ms, 1), "unit": "ms/step", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(), "host_cpus_available": avail,
            "stages_ms": {k: round(1e3 * v, 1) for k, v in times.items()},
            "one_core_ms_est": round(1e3 * cpu, 1),
            "sample": (f"the whole step, not a sample: FP64 oracle over all {n} Gaussians and all {P} pixels of "
                       f"the {W}x{H} view ({len(vals)} tile pairs), forward and backward in the oracle's tile-restricted mode, {cores} forked "
                       f"processes; one_core_ms_est = summed process CPU time of the same run")}


def serving_bench(n_requests: int, warmup: int):
    """Eight resident scenes (0.2M..3M Gaussians), Poisson arrivals of
    forward-only renders at 800x800 / 1280x720 / 1920x1080 from random cameras
    on a radius-6 sphere.  The one-at-a-time capacity mu1 is measured first
    (back-to-back submissions); then both the one-at-a-time server and the
    continuous-batching server run at 0.5, 0.8, 1.0 and 1.5 x mu1, each with
    `warmup` requests that are not counted followed by `n_requests` counted."""
    from paper_2411_12788_amd import raster as R
    from paper_2411_12788_amd.serve import GpuExecutor, Server, drive, poisson_arrivals
    scenes = {}
    for k, n in enumerate(gs_inputs.SERVING_SCENE_SIZES):
        # resident in the library's spatial order (served images do not depend on it)
        scenes[k] = R.DeviceScene.from_numpy(gs_inputs.surface_scene(n, 500 + k)).in_spatial_order()[0]
    torch.cuda.synchronize()
    resident = sum(s.nbytes() for s in scenes.values())

    def requests(count, seed):
        g = gs_inputs.rng(seed)
        out = []
        for _ in range(count):
            sid = int(g.integers(0, len(scenes)))
            w, h = gs_inputs.SERVING_RESOLUTIONS[int(g.integers(0, 3))]
            d = g.normal(size=3)
            d /= np.linalg.norm(d)
            out.append((sid, gs_inputs.look_at(6.0 * d, (0, 0, 0), w, h)))
        return out

    budget = 24 << 30
    # one-at-a-time capacity (back-to-back submissions, after a warm-up)
    ex1 = GpuExecutor(scenes, slots=1)
    srv = Server(ex1, budget, slots=1, max_batch=1)
    cap_n = max(40, n_requests // 4)
    cap = drive(srv, requests(warmup + cap_n, 2), [0.0] * (warmup + cap_n), warmup=warmup)
    srv.close()
    mu1 = cap["views_per_s"]
    out = {"workload": "8 resident scenes 0.2M-3M Gaussians (13.7M total), resolutions "
                       "800x800/1280x720/1920x1080, Poisson arrivals",
           "resident_gb": round(resident / 1e9, 3), "one_at_a_time_capacity_views_per_s": round(mu1, 2),
           "requests_per_point": n_requests, "warmup_per_point": warmup, "runs": []}
    for mode, slots, mb in (("one_at_a_time", 1, 1), ("continuous_batching", 4, 8)):
        for factor in (0.5, 0.8, 1.0, 1.5):
            ex = GpuExecutor(scenes, slots=slots)
            srv = Server(ex, budget, slots=slots, max_batch=mb)
            qps = factor * mu1
            total = warmup + n_requests
            seed = int(10 * factor) + 100 * slots
            st = drive(srv, requests(total, seed), poisson_arrivals(qps, total, seed + 1), warmup=warmup)
            srv.close()
            out["runs"].append({"mode": mode, "load": factor, "offered_qps": round(qps, 2),
                                "views_per_s": round(st["views_per_s"], 2), "p50_ms": round(st["p50_ms"], 3),
                                "p99_ms": round(st["p99_ms"], 3), "mean_ms": round(st["mean_ms"], 3),
                                "mean_batch": round(st["mean_batch"], 3), "batch_size_counts": st["batch_size_counts"],
                                "peak_reserved_gb": round(st["peak_reserved_gb"], 3), "requests": st["completed"],
                                "service_ms_by_batch": st["service_ms_by_batch"]})
    return out


def multiview_bench(steps: int, warmup: int):
    """Batched differentiation: one launch per stage for 16 views of a 1M-Gaussian
    scene at mixed resolutions (640x480 .. 1600x1200), forward + backward
    through the autograd Function, L1 loss; with recompute-in-backward (the
    default, least memory) and with the forward's lists kept (save_lists)."""
    from paper_2411_12788_amd import raster as R
    from paper_2411_12788_amd.autograd import rasterize
    wl = gs_inputs.multiview()
    sc = R.DeviceScene.from_numpy(wl.scene).in_spatial_order()[0]
    leaves = [t.clone().requires_grad_(True) for t in (sc.means, sc.scales, sc.quats, sc.opacity, sc.sh)]
    lay = R.view_layout(wl.cameras)
    target = torch.from_numpy(gs_inputs.uniform_image(3, lay.pixels_total, 777)).cuda()

    def run(save_lists):
        def one():
            for x in leaves:
                x.grad = None
            color, depth, imax = rasterize(*leaves, wl.cameras, save_lists=save_lists)
            (color - target).abs().mean().backward()

        for _ in range(warmup):
            one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            one()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / steps

    ms = run(False)
    ms_saved = run(True)
    return {"workload": wl.name, "gaussians": wl.scene.n, "views": len(wl.cameras),
            "pixels": lay.pixels_total, "ms_per_step": round(ms, 3), "views_per_s": round(1e3 * len(wl.cameras) / ms, 2),
            "mode": "autograd, recompute in backward",
            "saved_lists": {"ms_per_step": round(ms_saved, 3), "views_per_s": round(1e3 * len(wl.cameras) / ms_saved, 2)}}


def source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2411_12788_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


COUNTERS_MD = os.path.join(ROOT, "profiles", "counters_surfaces_3M_1920x1080.md")


def profile_counters():
    """Per-kernel counters of the committed summary (mean per dispatch), or {}
    when there is none or the kernel sources changed since it was taken."""
    if not os.path.exists(COUNTERS_MD):
        return {}
    txt = open(COUNTERS_MD).read()
    h = re.search(r"source_sha256:\s*([0-9a-f]+)", txt)
    if not h or h.group(1) != source_hash():
        return {}
    out = {}
    for m in re.finditer(r"^counters\[(k_[a-z0-9_]+)\]: (\{.*\})$", txt, flags=re.M):
        out[m.group(1)] = json.loads(m.group(2))
    return out


def profile_run(steps: int):
    """The profiled program: set-up (scene upload and its spatial order), then
    three 1 GiB device copies (the counters' calibration, and the marker after
    which every dispatch belongs to the steps), then `steps` steps."""
    wl = workload("large")
    step = Step(wl)
    torch.cuda.synchronize()
    a = torch.empty(1 << 28, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)  # 1 GiB read + 1 GiB written: calibration for the HBM counters
    torch.cuda.synchronize()
    copy_bytes = a.numel() * a.element_size()
    del a, b
    for _ in range(steps):
        step.run(record=False)
    torch.cuda.synchronize()
    print(json.dumps({"profile_steps": steps, "copy_bytes_each_way": copy_bytes, "source_sha256": source_hash()}),
          flush=True)


# rocprofv3 runs whose output `--summarize DIR` turns into profiles/ (one
# counter pass per run, within the per-block limits of one pass)
PROFILE_CMDS = {
    "kt": "rocprofv3 --kernel-trace --stats -d {d}/kt -o kt --output-format csv -- python3 bench.py --profile --steps 3",
    "fetch": "rocprofv3 --pmc FETCH_SIZE -d {d}/fetch -o fetch --output-format csv -- "
             "python3 bench.py --profile --steps 2",
    "write": "rocprofv3 --pmc WRITE_SIZE -d {d}/write -o write --output-format csv -- "
             "python3 bench.py --profile --steps 2",
    "dram": "rocprofv3 --pmc TCC_EA0_RDREQ_DRAM_32B_sum TCC_EA0_WRREQ_WRITE_DRAM_32B_sum "
            "TCC_EA0_WRREQ_ATOMIC_DRAM_32B_sum -d {d}/dram -o dram --output-format csv -- "
            "python3 bench.py --profile --steps 2",
    "sq": "rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_SALU SQ_INSTS_VMEM_RD SQ_WAVES SQ_ACTIVE_INST_VALU "
          "SQ_LDS_BANK_CONFLICT GRBM_GUI_ACTIVE -d {d}/sq -o sq --output-format csv -- "
          "python3 bench.py --profile --steps 2",
    "util": "rocprofv3 --pmc VALUBusy VALUUtilization LDSBankConflict MemUnitStalled -d {d}/util -o util "
            "--output-format csv -- python3 bench.py --profile --steps 2",
}
COPY_KERNEL = "copyBuffer (hipMemcpy D2D)"


def _short(name: str) -> str:
    m = re.search(r"msplat::(k_[a-z0-9_]+)", name)
    if m:
        return m.group(1)
    if "copyBuffer" in name:
        return COPY_KERNEL
    return name.split("(")[0][:60]


def summarize(d: str) -> None:
    """Turn the rocprofv3 runs of PROFILE_CMDS (sub-folders of d) into the text
    summaries kept under profiles/: kernel times, and per kernel the mean per
    dispatch of every counter collected.  HBM bytes per launch: FETCH_SIZE and
    WRITE_SIZE scaled by what they read for a 1 GiB copy ('traffic'), and the
    DRAM-bound 32-byte request counts times 32 ('dram')."""
    import csv
    dd = d.rstrip("/")
    # the sources the profiled runs were built from (written beside the runs'
    # output), else the current ones
    sha_file = os.path.join(d, "source_sha256.txt")
    sha = open(sha_file).read().strip() if os.path.exists(sha_file) else source_hash()

    def of_steps(rows, name_key):
        # the calibration copies (1 GiB each, the only copies of 100 us or
        # more) and every dispatch after the last of them (the steps); the
        # set-up before them (upload, spatial order) is left out
        rows = list(rows)

        def calib(r):
            return (_short(r[name_key]) == COPY_KERNEL and
                    int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) >= 100_000)
        marks = [int(r["Dispatch_Id"]) for r in rows if calib(r)]
        last = max(marks) if marks else -1
        return [r for r in rows if int(r["Dispatch_Id"]) > last or calib(r)]

    trace = of_steps(csv.DictReader(open(os.path.join(d, "kt", "kt_kernel_trace.csv"))), "Kernel_Name")
    durs = {}
    for r in trace:
        durs.setdefault(_short(r["Kernel_Name"]), []).append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in durs.values()) or 1.0
    lines = ["# Kernel times: 3M Gaussians, one 1920x1080 view, fwd+bwd step", "",
             "Command (from the repository root): `" + PROFILE_CMDS["kt"].format(d=dd) + "`", "",
             "From the kernel trace: the three calibration copies and every dispatch after them "
             "(the steps); the set-up before them (scene upload and spatial order) is left out.", "",
             f"source_sha256: {sha}", "",
             "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for k in sorted(durs, key=lambda x: -sum(durs[x])):
        v = durs[k]
        lines.append(f"| {k} | {len(v)} | {sum(v) / len(v):.1f} | {min(v):.1f} | {max(v):.1f} | "
                     f"{100.0 * sum(v) / total:.2f} |")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    open(os.path.join(ROOT, "profiles", "kernels_surfaces_3M_1920x1080.md"), "w").write("\n".join(lines) + "\n")
    avg_us = {k: sum(v) / len(v) for k, v in durs.items()}
    calls = {k: len(v) for k, v in durs.items()}

    per = {}  # kernel -> counter -> [values per dispatch]
    done = []
    for kind in PROFILE_CMDS:
        path = os.path.join(d, kind, f"{kind}_counter_collection.csv")
        if kind == "kt" or not os.path.exists(path):
            continue
        done.append(kind)
        for r in of_steps(csv.DictReader(open(path)), "Kernel_Name"):
            per.setdefault(_short(r["Kernel_Name"]), {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
    mean = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in per.items()}
    gib_kib = float(1 << 20)
    cp = mean.get(COPY_KERNEL, {})
    f_fac = max(per.get(COPY_KERNEL, {}).get("FETCH_SIZE", [gib_kib])) / gib_kib
    w_fac = max(per.get(COPY_KERNEL, {}).get("WRITE_SIZE", [gib_kib])) / gib_kib
    txt = ["# Counters per kernel: 3M Gaussians, one 1920x1080 view, fwd+bwd step", "",
           "Commands (from the repository root), one counter pass per run:", ""]
    txt += ["- `" + PROFILE_CMDS[k].format(d=dd) + "`" for k in ["kt"] + done]
    txt += ["", f"Calibration: a 1 GiB device copy reads {f_fac:.4f} GiB by FETCH_SIZE and writes {w_fac:.4f} GiB "
                f"by WRITE_SIZE; 'traffic' divides the two counters by these factors.  'dram' is 32 B x the "
                f"32-byte read, write and atomic requests the L2 sends to DRAM (no calibration; the copy reads "
                f"{32 * cp.get('TCC_EA0_RDREQ_DRAM_32B_sum', 0) / 2 ** 30:.3f} GiB and writes "
                f"{32 * cp.get('TCC_EA0_WRREQ_WRITE_DRAM_32B_sum', 0) / 2 ** 30:.3f} GiB by it).  VALU lane-ops "
                f"= 64 x SQ_INSTS_VALU (wave64 instructions issued).", "",
           "| kernel | calls | avg us | traffic MB | dram MB | GB/s (traffic) | VALU instr (M) | LDS instr (M) | "
           "VALUBusy % | VALUUtil % | LDS bank conflict % | mem stalled % |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    machine = []
    for k in sorted(mean, key=lambda x: -avg_us.get(x, 0.0)):
        c = mean[k]
        rec = {"avg_us": avg_us.get(k), "calls": calls.get(k)}
        if "FETCH_SIZE" in c and "WRITE_SIZE" in c:
            rec["traffic_bytes"] = 1024.0 * (c["FETCH_SIZE"] / f_fac + c["WRITE_SIZE"] / w_fac)
        if "TCC_EA0_RDREQ_DRAM_32B_sum" in c:
            rec["dram_read_bytes"] = 32.0 * c["TCC_EA0_RDREQ_DRAM_32B_sum"]
            rec["dram_write_bytes"] = 32.0 * (c.get("TCC_EA0_WRREQ_WRITE_DRAM_32B_sum", 0.0) +
                                             c.get("TCC_EA0_WRREQ_ATOMIC_DRAM_32B_sum", 0.0))
        rec.update({n: c[n] for n in c})
        machine.append(f"counters[{k}]: " + json.dumps(rec, sort_keys=True))
        us = avg_us.get(k, float("nan"))
        tr = rec.get("traffic_bytes")
        dr = (rec["dram_read_bytes"] + rec["dram_write_bytes"]) if "dram_read_bytes" in rec else None

        def f(x, scale=1.0, fmt="{:.1f}"):
            return fmt.format(x * scale) if x is not None else "-"
        txt.append(f"| {k} | {calls.get(k, '-')} | {us:.1f} | {f(tr, 1e-6)} | {f(dr, 1e-6)} | "
                   f"{f(tr / (us * 1e-6) / 1e9 if tr and us == us else None)} | {f(c.get('SQ_INSTS_VALU'), 1e-6, '{:.2f}')} | "
                   f"{f(c.get('SQ_INSTS_LDS'), 1e-6, '{:.2f}')} | {f(c.get('VALUBusy'))} | {f(c.get('VALUUtilization'))} | "
                   f"{f(c.get('LDSBankConflict'))} | {f(c.get('MemUnitStalled'))} |")
    txt += ["", "Machine-readable (mean per dispatch):", ""] + machine + ["", f"source_sha256: {sha}", ""]
    open(COUNTERS_MD, "w").write("\n".join(txt))
    print(f"wrote profiles/ from {d}")


def main():
    args = parse()
    if args.summarize:
        summarize(args.summarize)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only; multi-GPU runs are not implemented "
                                   "(the path would shard by view with a gradient all-reduce)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.profile:
        profile_run(max(2, args.steps))
        return
    wl = workload(args.workload)
    step = Step(wl, spatial=not args.input_order)
    for _ in range(args.warmup):
        step.run(record=False)
    step.prepare_events(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step.run(record=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    # the stage breakdown: the same number of steps again, with HIP events
    # around every stage (twelve more packets per step on the stream)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step.run(record=True)
    torch.cuda.synchronize()
    ms_step_events = 1e3 * (time.perf_counter() - t0) / args.steps
    step.collect()
    # the same step with the backward re-deriving projection and lists
    for _ in range(2):
        step.run(record=False, recompute=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step.run(record=False, recompute=True)
    torch.cuda.synchronize()
    ms_recompute = 1e3 * (time.perf_counter() - t1) / args.steps
    step.run(record=False)  # leave the kept-lists state for the figures below
    torch.cuda.synchronize()
    # the same workload with the Gaussians in their generated order, and the
    # one-off cost of the reorder
    other = Step(wl, spatial=args.input_order)
    for _ in range(args.warmup):
        other.run(record=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        other.run(record=False)
    torch.cuda.synchronize()
    ms_other = 1e3 * (time.perf_counter() - t2) / args.steps
    reorder_ms = spatial_order_ms(step if args.input_order else other)
    del other
    torch.cuda.empty_cache()
    med = {k: float(np.median(v)) for k, v in step.times.items()}
    avg = {k: float(np.mean(v)) for k, v in step.times.items()}
    st = step.stats
    n, P = step.n, step.lay.pixels_total
    nc = step.frame.n_contrib.double().sum().item()
    act_frac = float(step.active.float().mean().item()) if step.active is not None else 1.0
    n_vis = int(st.n_visible)
    n_act = int(step.active.sum().item()) if step.active is not None else n
    ev_fwd, ev_bwd = pair_evaluations(step)
    ni, nrec, tiles = int(st.n_isect), n * len(wl.cameras), int(st.tiles_total)
    passes = (int(st.key_bits) + 7) // 8
    ibits = max(1, (nrec - 1).bit_length())
    pair_pass = 16 if int(st.key_bits) + ibits <= 64 else 24
    # algorithmic bytes per step of each stage (the per-unit figures above times the units)
    alg = {
        "project": n_vis * PROJECT_BYTES_PER_RECORD + (n - n_vis) * PROJECT_BYTES_PER_UNDRAWN,
        "bin": nrec * 20 + (nrec * 20 + ni * 8 + ni * 8 + passes * pair_pass * ni + ni * 12 + tiles * 20),
        "render_fwd": ni * RENDER_FWD_BYTES_PER_PAIR + P * RENDER_FWD_BYTES_PER_PIXEL,
        "loss": P * 3 * 12,
        "render_bwd": ni * RENDER_BWD_BYTES_PER_PAIR + P * RENDER_BWD_BYTES_PER_PIXEL + ni * act_frac * 36,
        "project_bwd": n_act * PROJECT_BWD_BYTES_PER_ACTIVE + (n - n_act) * PROJECT_BWD_BYTES_PER_INACTIVE,
    }
    cnt = profile_counters()
    kt_steps = 3  # steps of the kernel-trace profile run (PROFILE_CMDS["kt"])
    stages = {}
    for k in step.names:
        a = alg[k] / (avg[k] * 1e-3) / 1e9
        e = {"ms": round(avg[k], 4), "bytes_algorithmic": int(alg[k]), "gbs_algorithmic": round(a, 1),
             "frac_hbm_algorithmic": round(a / PEAK_HBM_GBS, 4)}
        ks = [x for x in STAGE_KERNELS[k] if x in cnt]
        if ks:
            per_step = {x: (cnt[x].get("calls") or kt_steps) / kt_steps for x in ks}
            kus = sum(cnt[x]["avg_us"] * per_step[x] for x in ks if cnt[x].get("avg_us"))
            e["kernel_us_profiled"] = round(kus, 1)
            tr = [cnt[x].get("traffic_bytes") for x in ks]
            if all(t is not None for t in tr):
                tb = sum(t * per_step[x] for t, x in zip(tr, ks))
                e["traffic_bytes"] = int(tb)
                e["traffic_over_algorithmic"] = round(tb / alg[k], 3)
            dr = [cnt[x].get("dram_read_bytes") for x in ks]
            if all(t is not None for t in dr):
                e["dram_bytes"] = int(sum((cnt[x]["dram_read_bytes"] + cnt[x]["dram_write_bytes"]) * per_step[x]
                                          for x in ks))
            if k in ("render_fwd", "render_bwd") and "SQ_INSTS_VALU" in cnt[ks[0]]:
                lane_ops = 64.0 * cnt[ks[0]]["SQ_INSTS_VALU"]
                e["valu_lane_ops"] = lane_ops
                e["valu_tops"] = round(lane_ops / (avg[k] * 1e-3) / 1e12, 3)
                e["frac_valu"] = round(lane_ops / (avg[k] * 1e-3) / 1e12 / PEAK_VALU_TOPS, 4)
                for m in ("VALUBusy", "VALUUtilization", "LDSBankConflict", "MemUnitStalled"):
                    if m in cnt[ks[0]]:
                        e[m] = round(cnt[ks[0]][m], 2)
        stages[k] = e
    # the binning stage (pair count, its read-back, key emission, sort, ranges,
    # tile order): its algorithmic bytes over the profiled kernel time too, and
    # the profiled time of the count and the sort kernels apart
    kb = stages["bin"].get("kernel_us_profiled")
    if kb:
        stages["bin"]["frac_hbm_algorithmic_kernel_time"] = round(alg["bin"] / (kb * 1e-6) / 1e9 / PEAK_HBM_GBS, 4)
        for part, ks in BIN_PARTS.items():
            ks = [x for x in ks if x in cnt]
            stages["bin"][f"{part}_kernel_us_profiled"] = round(
                sum(cnt[x]["avg_us"] * (cnt[x].get("calls") or kt_steps) / kt_steps for x in ks), 1)
    dom = max(("project", "render_fwd", "render_bwd", "project_bwd"), key=lambda k: avg[k])
    sd = stages[dom]
    if dom in ("render_fwd", "render_bwd"):
        roof = {"bound": "alu", "kernel": STAGE_KERNELS[dom][0], "achieved": sd.get("valu_tops"),
                "peak": PEAK_VALU_TOPS, "unit": "T VALU lane-op/s", "frac": sd.get("frac_valu"),
                "hbm_gbs_algorithmic": sd["gbs_algorithmic"], "hbm_frac_algorithmic": sd["frac_hbm_algorithmic"]}
    else:
        roof = {"bound": "hbm", "kernel": STAGE_KERNELS[dom][0], "achieved": sd["gbs_algorithmic"],
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": sd["frac_hbm_algorithmic"]}
    roof["traffic"] = sd.get("traffic_bytes")
    roof["dram_bytes"] = sd.get("dram_bytes")
    roof["traffic_over_algorithmic"] = sd.get("traffic_over_algorithmic")
    for m in ("VALUBusy", "VALUUtilization", "LDSBankConflict", "MemUnitStalled"):
        if m in sd:
            roof[m] = sd[m]
    out = {
        "metric": "fwd+bwd ms/step @3M Gaussians 1080p; served views/s + p50/p99 latency",
        "value": round(ms_step, 4),
        "unit": "ms/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_recompute": round(ms_recompute, 4),
        "ms_per_step_with_stage_events": round(ms_step_events, 4),
        ("ms_per_step_spatial_order" if args.input_order else "ms_per_step_input_order"): round(ms_other, 4),
        "spatial_order_ms": round(reorder_ms, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "gaussians": n, "views": len(wl.cameras),
                   "resolution": f"{wl.cameras[0].width}x{wl.cameras[0].height}", "active_fraction": act_frac,
                   "layout": ("generated order" if args.input_order else
                              "spatial order (gs_spatial_order: the same Gaussians along the Morton curve)"),
                   "n_visible": n_vis, "n_isect": int(st.n_isect), "key_bits": int(st.key_bits),
                   "included_pairs": int(nc), "pair_evaluations_fwd": int(ev_fwd),
                   "pair_evaluations_bwd": int(ev_bwd)},
        "roofline": roof,
        "stages": stages,
    }
    out["stages"]["render_bwd_deterministic"] = {"ms": round(deterministic_backward_ms(step), 4)}
    out["stages"]["bin"]["sort_ms_by_pass_algorithm"] = {"prescan": round(bin_sort_ms(step, 0), 4),
                                                         "lookback": round(bin_sort_ms(step, 1), 4)}
    if not args.no_criteria:
        out["criteria"] = criteria_bench(step)
    if not args.no_multiview:
        out["multiview"] = multiview_bench(5, 2)
    if not args.no_serving:
        out["serving"] = serving_bench(args.serving_requests, args.serving_warmup)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_cores)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
