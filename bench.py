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
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import gs_inputs  # noqa: E402

PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
# algorithmic work per unit (measurement section)
FLOPS_FWD_PER_PAIR = 26.0          # alpha, transmittance, colour, argmax per included (pixel, Gaussian)
FLOPS_BWD_RECOMPUTE_PER_PAIR = 20.0  # alpha recompute, transmittance restore, suffix colour
FLOPS_BWD_GRAD_PER_PAIR = 35.0       # the nine partial derivatives of an active pair
PROJECT_BYTES_PER_RECORD = 59 * 4 + 64 + 16     # params read, record + bin written
PROJECT_BWD_BYTES_PER_ACTIVE = 59 * 4 + 59 * 4 + 36 + 16  # params read, grads written, 2D grad + bin read
PROJECT_BWD_BYTES_PER_INACTIVE = 59 * 4 + 1     # zero rows written, mask read


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large", choices=["large", "training", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-pixels", type=int, default=48)
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

    def __init__(self, wl):
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
        self.dldc = torch.empty((3, P), device="cuda")
        self.loss = torch.zeros(1, device="cuda")
        self.acc = R.alloc_accum(self.n)
        self.grads = R.alloc_grads(self.n)
        self.grad2d = torch.empty((self.n * len(self.cams), 9), device="cuda")
        self.names = ["project", "bin_count", "bin_sort", "render_fwd", "loss", "render_bwd", "project_bwd"]
        self.ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for k in self.names}
        self.times = {k: [] for k in self.names}
        self.frame = None

    def run(self, record: bool):
        R, ev = self.R, self.ev

        def mark(k, i):
            if record:
                ev[k][i].record()

        mark("project", 0)
        proj = R.project(self.scene, self.cams, self.opts)
        mark("project", 1)
        mark("bin_count", 0)
        offsets, st = R.bin_count(proj, self.cams, self.n)
        mark("bin_count", 1)
        mark("bin_sort", 0)
        binned = R.bin_sort(proj, self.cams, self.n, offsets, st)
        mark("bin_sort", 1)
        for t in self.acc.values():
            t.zero_()
        mark("render_fwd", 0)
        self.frame = R.render_forward(self.scene, proj, binned, self.cams, self.opts, accum=self.acc,
                                      extras=True, out=self.frame)
        mark("render_fwd", 1)
        self.loss.zero_()
        mark("loss", 0)
        R.l1_loss_grad(self.frame.color, self.target, self.dldc, self.loss)
        mark("loss", 1)
        self.grad2d.zero_()
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
        self.stats = st
        self.proj = proj

    def collect(self):
        torch.cuda.synchronize()
        for k in self.names:
            self.times[k].append(self.ev[k][0].elapsed_time(self.ev[k][1]))


def cpu_baseline(wl, sample_pixels: int):
    """The FP64 oracle on a bounded sample of the same step, scaled to ms/step."""
    import oracle
    cam = wl.cameras[0]
    p = oracle.Params.of(wl.scene)
    opts = oracle.Opts()
    t0 = time.perf_counter()
    proj = oracle.project(p, cam, opts)
    t1 = time.perf_counter()
    ordr = oracle.order(proj)
    t2 = time.perf_counter()
    g = gs_inputs.rng(99)
    pix = np.stack([g.integers(0, cam.width, sample_pixels), g.integers(0, cam.height, sample_pixels)], 1)
    oracle.render(p, cam, proj, ordr, opts, pixels=pix)
    dldc = g.normal(size=(sample_pixels, 3)) / (cam.width * cam.height)
    g2d = oracle.render_backward(p, cam, proj, ordr, opts, dldc, pixels=pix)
    t3 = time.perf_counter()
    oracle.project_backward(p, cam, opts, proj, g2d)
    t4 = time.perf_counter()
    per_pixel = (t3 - t2) / sample_pixels
    P = cam.width * cam.height
    ms = 1e3 * ((t1 - t0) + (t2 - t1) + (t4 - t3) + per_pixel * P)
    return {"value": ms, "unit": "ms/step", "cores": 1, "kind": "oracle",
            "sample": (f"full FP64 projection, depth order and projection backward of all {wl.scene.n} Gaussians "
                       f"+ forward and backward of {sample_pixels} seeded pixels over every Gaussian; per-pixel "
                       f"time scaled to the {P} pixels of the view; measured {t4 - t0:.1f} s")}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; multi-GPU scaling is not implemented "
                                   "(the path would shard by view with a gradient all-reduce)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    torch.cuda.set_device(0)
    wl = workload(args.workload)
    step = Step(wl)
    for _ in range(args.warmup):
        step.run(record=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step.run(record=True)
        step.collect()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    med = {k: float(np.median(v)) for k, v in step.times.items()}
    avg = {k: float(np.mean(v)) for k, v in step.times.items()}
    st = step.stats
    n, P = step.n, step.lay.pixels_total
    nc = step.frame.n_contrib.double().sum().item()
    act_frac = float(step.active.float().mean().item()) if step.active is not None else 1.0
    n_vis = int(st.n_visible)
    n_act = int(step.active.sum().item()) if step.active is not None else n
    work = {
        "render_fwd": ("alu", nc * FLOPS_FWD_PER_PAIR / 1e12, "TFLOP/s", PEAK_FP32_TFLOPS),
        "render_bwd": ("alu", nc * (FLOPS_BWD_RECOMPUTE_PER_PAIR + act_frac * FLOPS_BWD_GRAD_PER_PAIR) / 1e12,
                       "TFLOP/s", PEAK_FP32_TFLOPS),
        "project": ("hbm", n * PROJECT_BYTES_PER_RECORD / 1e9, "GB/s", PEAK_HBM_GBS),
        "project_bwd": ("hbm", (n_act * PROJECT_BWD_BYTES_PER_ACTIVE + (n - n_act) * PROJECT_BWD_BYTES_PER_INACTIVE)
                        / 1e9, "GB/s", PEAK_HBM_GBS),
    }
    dom = max(work.keys(), key=lambda k: avg[k])
    bound, units, unit, peak = work[dom]
    achieved = units / (avg[dom] * 1e-3)
    stages = {k: {"ms": round(avg[k], 4)} for k in step.names}
    for k, (b, u, un, pk) in work.items():
        a = u / (avg[k] * 1e-3)
        stages[k].update({"bound": b, "achieved": round(a, 3), "unit": un, "frac": round(a / pk, 4)})
    out = {
        "metric": "fwd+bwd ms/step @3M Gaussians 1080p",
        "value": round(ms_step, 4),
        "unit": "ms/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "gaussians": n, "views": len(wl.cameras),
                   "resolution": f"{wl.cameras[0].width}x{wl.cameras[0].height}", "active_fraction": act_frac,
                   "n_visible": n_vis, "n_isect": int(st.n_isect), "key_bits": int(st.key_bits),
                   "included_pairs": int(nc)},
        "roofline": {"bound": bound, "kernel": dom, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                     "frac": round(achieved / peak, 5), "traffic": None},
        "stages": stages,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_pixels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
