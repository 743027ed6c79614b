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
PEAK_FP32_TFLOPS = 157.3
# algorithmic work per unit (measurement section)
# Render work is counted in pair-evaluations of the tile algorithm (a pixel
# evaluates the entries of its tile's list in depth order until it stops; the
# backward revisits them up to the pixel's last contributor): ~25 VALU
# lane-ops + 1 exp2 each forward, ~3x that backward.  The kernels skip most of
# these evaluations with exact ellipse culling; they still count as the work
# the algorithm defines.
FLOPS_FWD_PER_EVAL = 26.0
FLOPS_BWD_PER_EVAL = 75.0
STOP_T = 0.01  # a pixel with final transmittance >= 1e-4 / (1 - 0.99) never stopped
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
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=240)
    ap.add_argument("--no-multiview", action="store_true")
    ap.add_argument("--no-criteria", action="store_true")
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
        self.bin_buffers = R.BinBuffers()

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
        # clears that the step needs anyway, queued while the host prepares the
        # sort launches (the pair count above is read back by the host)
        for t in self.acc.values():
            t.zero_()
        self.loss.zero_()
        self.grad2d.zero_()
        mark("bin_sort", 0)
        binned = R.bin_sort(proj, self.cams, self.n, offsets, st, buffers=self.bin_buffers)
        mark("bin_sort", 1)
        mark("render_fwd", 0)
        self.frame = R.render_forward(self.scene, proj, binned, self.cams, self.opts, accum=self.acc,
                                      extras=True, out=self.frame)
        mark("render_fwd", 1)
        mark("loss", 0)
        R.l1_loss_grad(self.frame.color, self.target, self.dldc, self.loss)
        mark("loss", 1)
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
        self.binned = binned

    def collect(self):
        torch.cuda.synchronize()
        for k in self.names:
            self.times[k].append(self.ev[k][0].elapsed_time(self.ev[k][1]))


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


def serving_bench(n_requests: int):
    """Eight resident scenes (0.2M..3M Gaussians), Poisson arrivals of
    forward-only renders at 800x800 / 1280x720 / 1920x1080 from random cameras
    on a radius-6 sphere.  One-at-a-time capacity mu1 is measured first; the
    continuous-batching server then runs at 0.8 and 1.5 x mu1, and the
    one-at-a-time server at 0.8 x mu1 for comparison."""
    from paper_2411_12788_amd import raster as R
    from paper_2411_12788_amd.serve import GpuExecutor, Server, drive, poisson_arrivals
    t_gen = time.perf_counter()
    scenes = {}
    for k, n in enumerate(gs_inputs.SERVING_SCENE_SIZES):
        scenes[k] = R.DeviceScene.from_numpy(gs_inputs.surface_scene(n, 500 + k))
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
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
    # warm-up and one-at-a-time capacity (back-to-back submissions)
    ex1 = GpuExecutor(scenes, slots=1)
    srv = Server(ex1, budget, slots=1, max_batch=1)
    drive(srv, requests(24, 1), [0.0] * 24)
    srv.close()
    srv = Server(ex1, budget, slots=1, max_batch=1)
    cap = drive(srv, requests(max(40, n_requests // 4), 2), [0.0] * max(40, n_requests // 4))
    srv.close()
    mu1 = cap["views_per_s"]
    out = {"workload": "8 resident scenes 0.2M-3M Gaussians (13.7M total), resolutions "
                       "800x800/1280x720/1920x1080, Poisson arrivals",
           "resident_gb": round(resident / 1e9, 3), "one_at_a_time_capacity_views_per_s": round(mu1, 2),
           "runs": []}
    for mode, slots, mb, factor in (("one_at_a_time", 1, 1, 0.8), ("continuous_batching", 4, 8, 0.8),
                                    ("continuous_batching", 4, 8, 1.5)):
        ex = GpuExecutor(scenes, slots=slots)
        srv = Server(ex, budget, slots=slots, max_batch=mb)
        qps = factor * mu1
        st = drive(srv, requests(n_requests, 10 + slots), poisson_arrivals(qps, n_requests, 20 + slots))
        srv.close()
        out["runs"].append({"mode": mode, "offered_qps": round(qps, 2), "views_per_s": round(st["views_per_s"], 2),
                            "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                            "mean_batch": round(st["mean_batch"], 2),
                            "peak_reserved_gb": round(st["peak_reserved_gb"], 3), "requests": st["completed"]})
    return out


def multiview_bench(steps: int, warmup: int):
    """Batched differentiation: one launch per stage for 16 views of a 1M-Gaussian
    scene at mixed resolutions (640x480 .. 1600x1200), forward + backward
    through the autograd Function, L1 loss; with recompute-in-backward (the
    default, least memory) and with the forward's lists kept (save_lists)."""
    from paper_2411_12788_amd import raster as R
    from paper_2411_12788_amd.autograd import rasterize
    wl = gs_inputs.multiview()
    sc = R.DeviceScene.from_numpy(wl.scene)
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


def traffic_from_profiles(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    h = re.search(r"source_sha256:\s*([0-9a-f]+)", txt)
    if not m or not h or h.group(1) != source_hash():
        return None
    return float(m.group(1))


def profile_run(steps: int):
    wl = workload("large")
    step = Step(wl)
    for _ in range(steps):
        step.run(record=False)
    torch.cuda.synchronize()
    a = torch.empty(1 << 28, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)  # 1 GiB read + 1 GiB written: calibration for the HBM counters
    torch.cuda.synchronize()
    print(json.dumps({"profile_steps": steps, "copy_bytes_each_way": a.numel() * 4, "source_sha256": source_hash()}),
          flush=True)


STAGE_KERNELS = {"render_fwd": "k_render_fwd", "render_bwd": "k_render_bwd", "project": "k_project",
                 "project_bwd": "k_project_bwd", "sort_pass": "k_os_pass"}
PROFILE_CMDS = {
    "kt": "rocprofv3 --kernel-trace --stats -d {d}/kt -o kt --output-format csv -- python3 bench.py --profile --steps 3",
    "fetch": "rocprofv3 --pmc FETCH_SIZE -d {d}/fetch -o fetch --output-format csv -- python3 bench.py --profile --steps 2",
    "write": "rocprofv3 --pmc WRITE_SIZE -d {d}/write -o write --output-format csv -- python3 bench.py --profile --steps 2",
}


def _short(name: str) -> str:
    m = re.search(r"msplat::(k_[a-z0-9_]+)", name)
    if m:
        return m.group(1)
    if "copyBuffer" in name:
        return "copyBuffer (hipMemcpy D2D)"
    return name.split("(")[0][:60]


def summarize(d: str) -> None:
    """Turn the three rocprofv3 runs of `bench.py --profile` into the text
    summaries kept under profiles/ (kernel times; HBM bytes per launch from
    FETCH_SIZE / WRITE_SIZE scaled by what the counters read for a 1 GiB copy)."""
    import csv
    stats = list(csv.DictReader(open(os.path.join(d, "kt", "kt_kernel_stats.csv"))))
    lines = ["# Kernel times: 3M Gaussians, one 1920x1080 view, fwd+bwd step", "",
             "Command (from the repository root): `" + PROFILE_CMDS["kt"].format(d=d.rstrip("/")) + "`", "",
             f"source_sha256: {source_hash()}", "",
             "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    open(os.path.join(ROOT, "profiles", "kernels_surfaces_3M_1920x1080.md"), "w").write("\n".join(lines) + "\n")

    def counter(kind):
        rows = list(csv.DictReader(open(os.path.join(d, kind, f"{kind}_counter_collection.csv"))))
        per = {}
        for r in rows:
            per.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        return per

    fetch, write = counter("fetch"), counter("write")
    copy = "copyBuffer (hipMemcpy D2D)"
    gib_kib = float(1 << 20)
    f_fac = max(fetch.get(copy, [gib_kib])) / gib_kib
    w_fac = max(write.get(copy, [gib_kib])) / gib_kib
    avg_us = {_short(r["Name"]): float(r["AverageNs"]) / 1e3 for r in stats}
    for stage, k in STAGE_KERNELS.items():
        if k not in fetch or k not in write:
            continue
        fk = sum(fetch[k]) / len(fetch[k])
        wk = sum(write[k]) / len(write[k])
        traffic = 1024.0 * (fk / f_fac + wk / w_fac)
        txt = [f"# HBM traffic of {k}: 3M Gaussians, one 1920x1080 view", "",
               "Commands (from the repository root):", "",
               "- `" + PROFILE_CMDS["fetch"].format(d=d.rstrip("/")) + "`",
               "- `" + PROFILE_CMDS["write"].format(d=d.rstrip("/")) + "`",
               "- `" + PROFILE_CMDS["kt"].format(d=d.rstrip("/")) + "` (durations)", "",
               f"- FETCH_SIZE per dispatch: {fk:.1f} KiB (mean of {len(fetch[k])} dispatches)",
               f"- WRITE_SIZE per dispatch: {wk:.1f} KiB",
               f"- calibration: a 1 GiB device copy reads {f_fac:.4f} GiB by FETCH_SIZE and writes "
               f"{w_fac:.4f} GiB by WRITE_SIZE; the counters are divided by these factors",
               f"- average duration: {avg_us.get(k, float('nan')):.1f} us",
               f"- measured HBM rate: {traffic / (avg_us.get(k, float('nan')) * 1e-6) / 1e9:.1f} GB/s", "",
               f"traffic_bytes_per_launch: {traffic:.6e}",
               f"source_sha256: {source_hash()}", ""]
        open(os.path.join(ROOT, "profiles", f"{stage}_counters.md"), "w").write("\n".join(txt))
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
    ev_fwd, ev_bwd = pair_evaluations(step)
    work = {
        "render_fwd": ("alu", ev_fwd * FLOPS_FWD_PER_EVAL / 1e12, "TFLOP/s", PEAK_FP32_TFLOPS),
        "render_bwd": ("alu", ev_bwd * FLOPS_BWD_PER_EVAL / 1e12, "TFLOP/s", PEAK_FP32_TFLOPS),
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
        "metric": "fwd+bwd ms/step @3M Gaussians 1080p; served views/s + p50/p99 latency",
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
                   "included_pairs": int(nc), "pair_evaluations_fwd": int(ev_fwd),
                   "pair_evaluations_bwd": int(ev_bwd)},
        "roofline": {"bound": bound, "kernel": dom, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                     "frac": round(achieved / peak, 5), "traffic": traffic_from_profiles(dom)},
        "stages": stages,
    }
    if not args.no_criteria:
        out["criteria"] = criteria_bench(step)
    if not args.no_multiview:
        out["multiview"] = multiview_bench(5, 2)
    if not args.no_serving:
        out["serving"] = serving_bench(args.serving_requests)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_pixels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
