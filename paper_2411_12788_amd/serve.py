"""Continuous-batching server for forward-only novel-view renders.

Scenes stay resident on the device.  Requests (scene, camera) arrive at any
time; a scheduler thread admits them while a slot (one HIP stream + one worker
thread) is free and their estimated HBM footprint fits the budget.  When a
slot frees up, the oldest waiting request is admitted together with the other
waiting requests for the same scene (up to ``max_batch`` views, any mix of
resolutions): they render in one multi-view launch per stage.  Work on
different slots overlaps on the GPU.  Admission is two-phase because the pair
count is only known after projection: a request first reserves an estimate,
and once the pairs are counted the executor grows (or shrinks) the reservation
to the real figure, waiting if the budget is momentarily full, before any of
the slot's buffers grow.

Latency is measured from arrival to completion of the request's last kernel
(host copy excluded).  ``Server`` is independent of the GPU; ``GpuExecutor``
drives libmsplat.so through ``raster``.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from concurrent.futures import Future
from typing import Any, Callable, Dict, List, Optional, Sequence


@dataclasses.dataclass
class Request:
    scene_id: Any
    camera: Any
    arrival: float = 0.0
    future: Future = dataclasses.field(default_factory=Future)
    seq: int = 0


@dataclasses.dataclass
class Result:
    color: Any            # [3, H, W] (device tensor for the GPU executor)
    depth: Any
    latency: float        # seconds, arrival -> completion
    batch_size: int
    slot: int


class AdmissionError(RuntimeError):
    pass


class Server:
    """Scheduler: FIFO queue, HBM-footprint admission, slots, scene-grouped batching."""

    def __init__(self, executor, hbm_budget: int, slots: int = 4, max_batch: int = 8,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_batch = max(1, int(max_batch))
        self.clock = clock
        self.cv = threading.Condition()
        self.queue: collections.deque = collections.deque()
        self.free_slots = list(range(slots))
        self.reserved = 0
        self.peak_reserved = 0
        self.in_flight = 0
        self.growing = 0
        self.slot_extra: Dict[int, int] = {}  # second-phase adjustment of each running batch
        self.completed: List[Result] = []
        self.service: List[Any] = []  # (batch size, seconds from admission to completion)
        self.admitted_batches: List[int] = []
        self.running = True
        self.seq = 0
        self.workers: Dict[int, threading.Thread] = {}
        self.sched = threading.Thread(target=self._schedule, daemon=True)
        self.sched.start()

    # -- client side -------------------------------------------------------
    def submit(self, scene_id, camera, arrival: Optional[float] = None) -> Future:
        req = Request(scene_id, camera, self.clock() if arrival is None else arrival)
        with self.cv:
            if not self.running:
                raise RuntimeError("server closed")
            req.seq = self.seq
            self.seq += 1
            self.queue.append(req)
            self.cv.notify_all()
        return req.future

    def drain(self, timeout: float = 600.0) -> None:
        end = time.monotonic() + timeout
        with self.cv:
            while self.queue or self.in_flight:
                left = end - time.monotonic()
                if left <= 0:
                    raise TimeoutError("drain timed out")
                self.cv.wait(timeout=min(left, 0.5))

    def close(self) -> None:
        with self.cv:
            self.running = False
            self.cv.notify_all()
        self.sched.join(timeout=5)
        for t in list(self.workers.values()):
            t.join(timeout=30)

    # -- reservations --------------------------------------------------------
    def grow(self, delta: int, slot: int, timeout: float = 60.0) -> None:
        """Second admission phase: adjust the reservation of the batch running
        on `slot`.  The adjustment is recorded per slot and released with the
        batch, whether or not the batch then completes.

        A batch that needs more memory waits while some other in-flight batch
        is still running (it will release memory); when every in-flight batch
        is itself waiting to grow, the request proceeds (the budget is then
        exceeded by at most the estimation error of the batches in flight)."""
        end = time.monotonic() + timeout
        with self.cv:
            if delta > 0:
                self.growing += 1
                try:
                    while self.reserved + delta > self.budget and self.in_flight - self.growing > 0:
                        left = end - time.monotonic()
                        if left <= 0:
                            raise AdmissionError("could not grow reservation in time")
                        self.cv.wait(timeout=min(left, 0.5))
                finally:
                    self.growing -= 1
            self.reserved += delta
            self.slot_extra[slot] = self.slot_extra.get(slot, 0) + delta
            self.peak_reserved = max(self.peak_reserved, self.reserved)
            self.cv.notify_all()

    # -- scheduler -----------------------------------------------------------
    def _pick(self):
        head = self.queue[0]
        batch = [head]
        for r in list(self.queue)[1:]:
            if len(batch) >= self.max_batch:
                break
            if r.scene_id == head.scene_id:
                batch.append(r)
        return batch

    def _schedule(self) -> None:
        while True:
            with self.cv:
                while self.running and (not self.queue or not self.free_slots):
                    self.cv.wait(timeout=0.5)
                if not self.running and not self.queue:
                    return
                if not self.queue or not self.free_slots:
                    continue
                batch = self._pick()
                need = self.ex.footprint(batch)
                while need > self.budget - self.reserved and len(batch) > 1:
                    batch = batch[:-1]
                    need = self.ex.footprint(batch)
                if need > self.budget - self.reserved:
                    if self.in_flight == 0:
                        # cannot ever fit: fail the request rather than wait forever
                        req = self.queue.popleft()
                        req.future.set_exception(AdmissionError(
                            f"request needs {need} B, budget is {self.budget} B"))
                        continue
                    self.cv.wait(timeout=0.5)
                    continue
                for r in batch:
                    self.queue.remove(r)
                slot = self.free_slots.pop(0)
                self.reserved += need
                self.peak_reserved = max(self.peak_reserved, self.reserved)
                self.in_flight += 1
                self.admitted_batches.append(len(batch))
                t = threading.Thread(target=self._work, args=(batch, slot, need), daemon=True)
                self.workers[slot] = t
                t.start()

    def _work(self, batch: List[Request], slot: int, reserved: int) -> None:
        start = self.clock()
        try:
            outs = self.ex.run(batch, slot, self)
            done = self.clock()
            results = []
            for r, (color, depth) in zip(batch, outs):
                res = Result(color, depth, done - r.arrival, len(batch), slot)
                results.append(res)
            err = None
        except BaseException as e:  # noqa: BLE001 - propagate to the futures
            err, results = e, []
            done = self.clock()
        with self.cv:
            self.reserved -= reserved + self.slot_extra.pop(slot, 0)
            self.in_flight -= 1
            self.free_slots.append(slot)
            # the server keeps the timing only: the frames are the clients'
            # (holding them here would keep every served frame on the device)
            self.completed.extend(Result(None, None, r.latency, r.batch_size, r.slot) for r in results)
            self.service.append((len(batch), done - start))
            self.cv.notify_all()
        if err is not None:
            for r in batch:
                if not r.future.done():
                    r.future.set_exception(err)
        else:
            for r, res in zip(batch, results):
                r.future.set_result(res)

    # -- metrics -------------------------------------------------------------
    def stats(self, t0: Optional[float] = None, t1: Optional[float] = None) -> Dict[str, float]:
        lat = sorted(r.latency for r in self.completed)
        if not lat:
            return {"completed": 0}
        n = len(lat)

        def pct(p):
            return lat[min(n - 1, int(round(p / 100.0 * (n - 1))))]

        out = {"completed": n, "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99), "mean_ms": 1e3 * sum(lat) / n,
               "mean_batch": sum(self.admitted_batches) / max(1, len(self.admitted_batches)),
               "peak_reserved_gb": self.peak_reserved / 1e9}
        if t0 is not None and t1 is not None and t1 > t0:
            out["views_per_s"] = n / (t1 - t0)
        return out


class GpuExecutor:
    """Runs a batch of same-scene views as one multi-view launch per stage on
    the slot's HIP stream."""

    def __init__(self, scenes: Dict[Any, Any], slots: int, opts=None, device: str = "cuda"):
        import torch

        from . import raster as R
        self.R = R
        self.torch = torch
        self.scenes = scenes  # scene_id -> raster.DeviceScene (resident)
        # tile culling at emission leaves every rendered output unchanged and
        # drops the pairs that cannot composite (~12 % on dense scenes)
        self.opts = opts or R.RasterOpts(tile_cull=True)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        # per slot: projection records, pair count and lists are reused from
        # batch to batch (a slot runs one batch at a time), so the allocator
        # is not asked for gigabytes of new blocks per batch; only the frames
        # handed to clients are allocated per batch
        self.buffers = [R.StepBuffers() for _ in range(slots)]
        self.pairs_per_record: Dict[Any, float] = {}
        self.lock = threading.Lock()

    # bytes held by one batch (records, lists, sort workspace, outputs)
    def _bytes(self, n: int, V: int, P: int, n_isect: int) -> int:
        rec = V * n * (64 + 16 + 4) + 8 * ((V * n) // 4096 + 1) * 8
        pairs = n_isect * (4 + 8 + 4 + 8 + 4) + (n_isect // 4096 + 1) * 256 * 4 * 2
        frame = P * (12 + 4 + 4 + 4 + 4)
        return int(rec + pairs + frame) + (1 << 20)

    def footprint(self, batch: Sequence[Request]) -> int:
        sid = batch[0].scene_id
        n = self.scenes[sid].n
        V = len(batch)
        P = sum(int(r.camera.width) * int(r.camera.height) for r in batch)
        ppr = self.pairs_per_record.get(sid, 2.0)
        return self._bytes(n, V, P, int(ppr * V * n))

    def run(self, batch: Sequence[Request], slot: int, server: Server):
        R, torch = self.R, self.torch
        sid = batch[0].scene_id
        scene = self.scenes[sid]
        cams = [r.camera for r in batch]
        st = self.streams[slot]
        with torch.cuda.stream(st):
            buf = self.buffers[slot]
            proj = R.project(scene, cams, self.opts, stream=st, buffers=buf)
            est = self.footprint(batch)

            def counted(stats):
                # second admission phase, before any buffer of the slot grows
                real = self._bytes(scene.n, len(cams), sum(c.width * c.height for c in cams), int(stats.n_isect))
                if real != est:
                    server.grow(real - est, slot)
                with self.lock:
                    ppr = stats.n_isect / max(1, len(cams) * scene.n)
                    old = self.pairs_per_record.get(sid)
                    self.pairs_per_record[sid] = ppr if old is None else max(ppr, 0.5 * (old + ppr))

            # count and sort in one library call when the slot's buffers hold
            # the pairs
            binned = R.bin_step(proj, cams, scene.n, buf, stream=st, on_count=counted)
            frame = R.render_forward(scene, proj, binned, cams, self.opts, extras=False, stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        ev.synchronize()
        outs = []
        off = 0
        for c in cams:
            m = int(c.width) * int(c.height)
            outs.append((frame.color[:, off:off + m].view(3, int(c.height), int(c.width)),
                         frame.depth[off:off + m].view(int(c.height), int(c.width))))
            off += m
        return outs


class FakeExecutor:
    """CPU stand-in with simulated durations and footprints (scheduler tests)."""

    def __init__(self, sizes: Dict[Any, int], per_view_s: float = 0.002, per_batch_s: float = 0.003,
                 bytes_per_gaussian: int = 100, realised_factor: float = 1.0, fail_after_grow: bool = False):
        self.sizes = sizes
        self.per_view_s = per_view_s
        self.per_batch_s = per_batch_s
        self.bpg = bytes_per_gaussian
        self.realised = realised_factor
        self.fail_after_grow = fail_after_grow
        self.max_concurrency = 0
        self.active = 0
        self.lock = threading.Lock()
        self.batches: List[List[int]] = []

    def footprint(self, batch):
        return self.sizes[batch[0].scene_id] * self.bpg * len(batch)

    def run(self, batch, slot, server):
        with self.lock:
            self.active += 1
            self.max_concurrency = max(self.max_concurrency, self.active)
            self.batches.append([r.seq for r in batch])
        try:
            if self.realised != 1.0:
                server.grow(int(self.footprint(batch) * (self.realised - 1.0)), slot)
                if self.fail_after_grow:
                    raise RuntimeError("simulated failure after the reservation grew")
            time.sleep(self.per_batch_s + self.per_view_s * len(batch))
        finally:
            with self.lock:
                self.active -= 1
        return [((r.scene_id, r.camera), None) for r in batch]


def poisson_arrivals(qps: float, count: int, seed: int) -> List[float]:
    import numpy as np
    g = np.random.Generator(np.random.PCG64(seed))
    return list(np.cumsum(g.exponential(1.0 / qps, size=count)))


def drive(server: Server, requests: Sequence, arrivals: Sequence[float], warmup: int = 0) -> Dict[str, Any]:
    """Submit ``requests`` [(scene_id, camera)] at the given offsets (seconds)
    from now, wait for all, and return latency / throughput statistics of the
    requests after the first ``warmup`` (which run but are not counted):
    p50 / p99 / mean latency, views/s over the window from the first counted
    arrival (or the last warm-up completion, if later) to the last counted
    completion, the offered rate, and the distribution of the batch sizes the
    counted requests were rendered in."""
    t0 = server.clock()
    # Results are read as they complete and not kept (a served frame is the
    # client's to consume; holding every frame until the end of a run would
    # keep the device memory of all of them alive).
    total = len(arrivals)
    recs: List[Any] = [None] * total
    lock = threading.Condition()
    left = [total]

    def collect(k):
        def done(f):
            try:
                r = f.result()
                rec = (r.latency, r.batch_size)
            except BaseException as e:  # noqa: BLE001 - reported below
                rec = e
            with lock:
                recs[k] = rec
                left[0] -= 1
                lock.notify_all()
        return done

    for k, ((sid, cam), a) in enumerate(zip(requests, arrivals)):
        now = server.clock() - t0
        if a > now:
            time.sleep(a - now)
        server.submit(sid, cam, arrival=t0 + a).add_done_callback(collect(k))
    with lock:
        end_wait = time.monotonic() + 600.0
        while left[0] > 0:
            rem = end_wait - time.monotonic()
            if rem <= 0:
                raise TimeoutError("requests did not complete")
            lock.wait(timeout=min(rem, 1.0))
    for r in recs:
        if isinstance(r, BaseException):
            raise r
    res = [Result(None, None, lat, bs, -1) for lat, bs in recs]
    w = max(0, min(int(warmup), len(res) - 1))
    meas, arr = res[w:], list(arrivals[w:])
    lat = sorted(r.latency for r in meas)
    n = len(lat)

    def pct(p):
        return lat[min(n - 1, int(round(p / 100.0 * (n - 1))))]

    # throughput window: from the first counted arrival, or from the last
    # warm-up completion if that is later (with every request submitted at
    # once, the counted ones wait for the warm-up to be served), to the last
    # counted completion
    done = max(a + r.latency for a, r in zip(arr, meas))
    start = arr[0]
    if w > 0:
        start = max(start, max(a + r.latency for a, r in zip(arrivals[:w], res[:w])))
    span = done - start
    sizes: Dict[int, int] = {}
    for r in meas:
        sizes[r.batch_size] = sizes.get(r.batch_size, 0) + 1
    st: Dict[str, Any] = {"completed": n, "warmup": w, "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99),
                          "mean_ms": 1e3 * sum(lat) / n, "mean_batch": sum(r.batch_size for r in meas) / n,
                          "batch_size_counts": {str(k): sizes[k] for k in sorted(sizes)},
                          "peak_reserved_gb": server.peak_reserved / 1e9,
                          "views_per_s": n / span if span > 0 else float("inf")}
    st["offered_qps"] = (len(arr) - 1) / max(arr[-1] - arr[0], 1e-9) if len(arr) > 1 else 0.0
    # admission-to-completion time of a batch, by its size (every batch of the
    # run, warm-up included): with several slots it includes the time the
    # batch shared the device with the others
    by: Dict[int, List[float]] = {}
    with server.cv:
        for bs, sec in server.service:
            by.setdefault(bs, []).append(sec)
    st["service_ms_by_batch"] = {str(k): round(1e3 * sum(v) / len(v), 3) for k, v in sorted(by.items())}
    return st
