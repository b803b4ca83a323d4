"""Render serving with the map resident in HBM: continuous batching of colour + depth queries
of mixed resolutions and poses, admitted against a device-memory budget, executed on several
streams so that batches overlap on the GPU; latency (completion - arrival) is recorded per
query and summarised as p50 / p99 beside throughput.

Structure
  * ``Request``: one query (intrinsics, pose) with arrival / completion timestamps.
  * ``Server``: an admission queue and ``n_slots`` worker threads.  The device-memory budget
    covers two things: each slot's workspace, sized once when the server starts (the largest
    batch whose workspace and outputs fit n_slots times in the budget) and charged for the
    server's lifetime; and the outputs (colour, depth, transmittance) of every admitted
    request, charged at admission and released at completion.  A worker that becomes free
    takes as many admitted requests as fit its batch limits and its slot's workspace (FIFO),
    launches them as one multi-view call on its own stream, waits for that stream only, then
    releases the memory and completes the requests.  Requests arriving while batches run are
    admitted as memory frees up, so work from different arrivals overlaps on the device.
    Completed outputs belong to the caller (``keep_outputs``) or are dropped.
  * ``GpuExecutor``: runs a batch through the C ABI (tsr_bin_and_sort + tsr_render_forward)
    on the worker's stream in the slot's fixed workspace; a batch whose pairs overflow it is
    split in halves.  ``FakeExecutor`` (tests) sleeps instead.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Callable, Deque, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    intr: object                  # scenes.Intrinsics
    pose: np.ndarray              # [12] float32 T_CW
    arrival: float = 0.0
    admitted: float = 0.0
    done: float = 0.0
    nbytes: int = 0
    color: object = None          # [3, H, W] device tensor after completion
    depth: object = None          # [H, W]
    error: Optional[str] = None
    event: threading.Event = dataclasses.field(default_factory=threading.Event)

    @property
    def pixels(self) -> int:
        return int(self.intr.width) * int(self.intr.height)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class FakeExecutor:
    """Scheduler tests: 'renders' by sleeping `per_pixel_s` per pixel; can inject failures."""

    def __init__(self, per_pixel_s: float = 1e-8, fail_ids: Sequence[int] = ()):
        self.per_pixel_s = per_pixel_s
        self.fail_ids = set(fail_ids)
        self.batches: List[List[int]] = []
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0

    def setup(self, n_slots: int, budget: int, max_views: int, max_pixels: int):
        return 0, max_views

    def batch_fits(self, intrs) -> bool:
        return True

    def request_error(self, req: Request) -> Optional[str]:
        return None

    def estimate_bytes(self, req: Request) -> int:
        return 20 * req.pixels

    def make_slot(self, i: int):
        return None

    def run(self, slot, batch: List[Request]) -> None:
        with self.lock:
            self.batches.append([r.rid for r in batch])
            self.active += 1
            self.max_active = max(self.max_active, self.active)
        try:
            time.sleep(self.per_pixel_s * sum(r.pixels for r in batch))
            for r in batch:
                if r.rid in self.fail_ids:
                    r.error = "injected failure"
        finally:
            with self.lock:
                self.active -= 1


class GpuExecutor:
    """Executes batches through the rasterizer on per-slot HIP streams, each slot with one
    workspace buffer sized when the server starts."""

    OUT_BYTES_PER_PIXEL = 20          # colour (12), depth (4), transmittance (4)

    def __init__(self, dev_scene, params=None, pairs_per_tile: float = 160.0, max_resolution=(1200, 680)):
        import torch

        from . import raster

        self.torch = torch
        self.raster = raster
        self.scene = dev_scene
        self.params = params or raster.Params()
        self.pairs_per_tile = pairs_per_tile          # capacity estimate, raised on overflow
        self.max_resolution = tuple(max_resolution)
        self.lock = threading.Lock()
        self.retries = 0
        self.slot_bytes = 0

    def _capacity(self, intrs) -> int:
        tiles = sum(((i.width + 15) // 16) * ((i.height + 15) // 16) for i in intrs)
        return int(self.pairs_per_tile * tiles) + 4096

    def _workspace_bytes(self, intrs, cap) -> int:
        import ctypes as C

        from ._lib import check, load

        out = C.c_size_t(0)
        sc = self.scene.c()
        check(load().tsr_workspace_size(C.byref(sc), self.raster.intrinsics_array(intrs), len(intrs), cap,
                                        C.byref(out)), "tsr_workspace_size")
        return int(out.value)

    def setup(self, n_slots: int, budget: int, max_views: int, max_pixels: int):
        """Slot workspace size: the largest batch of v <= max_views views at max_resolution
        whose workspace plus outputs fit n_slots times in the budget.  Returns (bytes the
        slots hold for the server's lifetime, v)."""
        from .scenes import intrinsics_for

        intr = intrinsics_for(*self.max_resolution)
        px = intr.width * intr.height
        for v in range(max(1, max_views), 0, -1):
            if v > 1 and v * px > max_pixels:
                continue
            ws = self.slot_workspace_bytes(v)
            if n_slots * (ws + v * px * self.OUT_BYTES_PER_PIXEL) <= budget:
                self.slot_bytes = ws
                return n_slots * ws, v
        raise ValueError(f"a budget of {budget} B cannot hold {n_slots} slot workspaces of one "
                         f"{intr.width}x{intr.height} view each")

    def slot_workspace_bytes(self, v: int) -> int:
        """Workspace of a slot for batches of v views at max_resolution: pair room for the batch
        at the estimated density, and for one view at four times it (a view close to a wall can
        list several times the average; pairs cost 16 B each)."""
        from .scenes import intrinsics_for

        intr = intrinsics_for(*self.max_resolution)
        cap = max(self._capacity([intr] * v), 4 * self._capacity([intr]))
        return self._workspace_bytes([intr] * v, cap)

    def batch_fits(self, intrs) -> bool:
        return self._workspace_bytes(intrs, self._capacity(intrs)) <= self.slot_bytes

    def request_error(self, req: Request) -> Optional[str]:
        if not self.batch_fits([req.intr]):
            return f"a {req.intr.width}x{req.intr.height} view needs more workspace than a slot's {self.slot_bytes} B"
        return None

    def estimate_bytes(self, req: Request) -> int:
        return self.OUT_BYTES_PER_PIXEL * req.pixels

    def make_slot(self, i: int):
        # a stream and the workspace buffer every batch of this slot reuses
        return {"stream": self.torch.cuda.Stream(),
                "ws": self.torch.empty(self.slot_bytes, dtype=self.torch.uint8, device="cuda")}

    def _render(self, slot, batch: List[Request]) -> None:
        torch, raster = self.torch, self.raster
        stream = slot["stream"]
        intrs = [r.intr for r in batch]
        if self._workspace_bytes(intrs, 0) > slot["ws"].numel():
            raise RuntimeError("batch does not fit the slot's workspace")
        rast = raster.Rasterizer(self.scene, intrs, self.params, workspace=slot["ws"])
        poses = raster.poses_tensor([r.pose for r in batch])
        rast.bin_and_sort(poses, stream=stream, check_capacity=False)
        color, depth, _ = rast.forward(poses, stream=stream)
        rc = rast.lib.tsr_check(raster._ptr(rast.ws), raster._stream(stream), None)   # syncs this stream
        if rc == raster._lib.TSR_ECAPACITY:
            # more pairs than the slot's buffer holds: raise the density estimate for later
            # batches and admission, and render the batch in halves
            k = rast.count(poses, stream=stream)
            tiles = sum(((i.width + 15) // 16) * ((i.height + 15) // 16) for i in intrs)
            with self.lock:
                self.retries += 1
                self.pairs_per_tile = max(self.pairs_per_tile, 1.1 * k / max(tiles, 1))
            if len(batch) == 1:
                raise RuntimeError(f"one view with {k} pairs does not fit a slot's workspace ({rast.capacity} pairs)")
            del rast, color, depth
            h = len(batch) // 2
            self._render(slot, batch[:h])
            self._render(slot, batch[h:])
            return
        raster.check(rc, "tsr_check")
        cs, ds = rast.split_views(color, 3), rast.split_views(depth, 1)
        for r, c, d in zip(batch, cs, ds):
            r.color, r.depth = c, d[0]

    def run(self, slot, batch: List[Request]) -> None:
        with self.torch.cuda.stream(slot["stream"]):
            self._render(slot, batch)


class Server:
    def __init__(self, executor, n_slots: int = 4, mem_budget: int = 8 << 30, max_batch_views: int = 8,
                 max_batch_pixels: int = 8 * 1200 * 680, clock: Callable[[], float] = time.perf_counter,
                 keep_outputs: bool = True):
        self.ex = executor
        self.n_slots = n_slots
        self.budget = mem_budget
        self.used = 0
        self.fixed = 0                  # slot workspaces, charged while the server runs
        self.keep_outputs = keep_outputs
        self.max_views = max_batch_views
        self.max_pixels = max_batch_pixels
        self.clock = clock
        self.cv = threading.Condition()
        self.waiting: Deque[Request] = collections.deque()     # arrived, not admitted
        self.ready: Deque[Request] = collections.deque()       # admitted, not launched
        self.completed: List[Request] = []
        self.stop_flag = False
        self.threads: List[threading.Thread] = []
        self.peak_used = 0
        self.inflight_batches = 0
        self.peak_inflight = 0

    # ------------------------------------------------------------------ public
    def start(self) -> None:
        fixed, views = self.ex.setup(self.n_slots, self.budget, self.max_views, self.max_pixels)
        with self.cv:
            self.fixed = int(fixed)
            self.max_views = min(self.max_views, int(views))
            self.used += self.fixed
            self.peak_used = max(self.peak_used, self.used)
        for i in range(self.n_slots):
            slot = self.ex.make_slot(i)
            t = threading.Thread(target=self._worker, args=(slot,), daemon=True)
            t.start()
            self.threads.append(t)

    def submit(self, req: Request) -> Request:
        req.arrival = self.clock()
        req.nbytes = self.ex.estimate_bytes(req)
        err = self.ex.request_error(req)
        with self.cv:
            if err is None and req.nbytes > self.budget - self.fixed:
                err = (f"request needs {req.nbytes} B, above the budget of {self.budget} B less the "
                       f"{self.fixed} B the slots hold")
            if err is not None:
                req.error = err
                req.done = self.clock()
                self.completed.append(req)
                req.event.set()
                return req
            self.waiting.append(req)
            self._admit_locked()
            self.cv.notify_all()
        return req

    def drain(self, timeout: float = 600.0) -> None:
        end = time.monotonic() + timeout
        with self.cv:
            while self.waiting or self.ready or self.inflight_batches:
                left = end - time.monotonic()
                if left <= 0:
                    raise TimeoutError("server did not drain")
                self.cv.wait(min(left, 0.05))

    def stop(self) -> None:
        with self.cv:
            self.stop_flag = True
            self.cv.notify_all()
        for t in self.threads:
            t.join(timeout=10)
        with self.cv:
            self.used -= self.fixed
            self.fixed = 0

    def stats(self) -> dict:
        ok = [r for r in self.completed if r.error is None]
        lat = np.array([r.latency for r in ok]) * 1e3
        if not ok:
            return {"completed": 0, "errors": len(self.completed)}
        span = max(r.done for r in ok) - min(r.arrival for r in ok)
        return {"completed": len(ok), "errors": len(self.completed) - len(ok), "samples": int(lat.size),
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "qps": len(ok) / span if span > 0 else float("nan"),
                "mpix_s": sum(r.pixels for r in ok) / span / 1e6 if span > 0 else float("nan"),
                "peak_mem": self.peak_used, "peak_inflight_batches": self.peak_inflight,
                "max_batch_views": self.max_views}

    # ------------------------------------------------------------------ internals
    def _admit_locked(self) -> None:
        while self.waiting and self.used + self.waiting[0].nbytes <= self.budget:
            r = self.waiting.popleft()
            self.used += r.nbytes
            self.peak_used = max(self.peak_used, self.used)
            r.admitted = self.clock()
            self.ready.append(r)

    def _take_batch_locked(self) -> List[Request]:
        batch, px = [], 0
        while self.ready and len(batch) < self.max_views:
            r = self.ready[0]
            if batch and (px + r.pixels > self.max_pixels or not self.ex.batch_fits([q.intr for q in batch + [r]])):
                break
            batch.append(self.ready.popleft())
            px += r.pixels
        return batch

    def _worker(self, slot) -> None:
        while True:
            with self.cv:
                while not self.ready and not self.stop_flag:
                    self.cv.wait(0.05)
                if self.stop_flag and not self.ready:
                    return
                batch = self._take_batch_locked()
                self.inflight_batches += 1
                self.peak_inflight = max(self.peak_inflight, self.inflight_batches)
            try:
                self.ex.run(slot, batch)
            except Exception as e:                         # a failed batch fails only its requests
                for r in batch:
                    r.error = f"{type(e).__name__}: {e}"
            now = self.clock()
            with self.cv:
                for r in batch:
                    r.done = now
                    if not self.keep_outputs:
                        r.color = r.depth = None
                    self.used -= r.nbytes
                    self.completed.append(r)
                    r.event.set()
                self.inflight_batches -= 1
                self._admit_locked()
                self.cv.notify_all()


def run_poisson(server: Server, queries, time_scale: float = 1.0, warmup: int = 0) -> dict:
    """Submit (arrival_s, intr, pose) queries at their Poisson arrival times; returns stats of
    the queries after the first `warmup`."""
    t0 = time.perf_counter()
    reqs = []
    for i, (t_arr, intr, pose) in enumerate(queries):
        delay = t0 + t_arr * time_scale - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        reqs.append(server.submit(Request(i, intr, pose)))
    server.drain()
    keep = {r.rid for r in reqs[warmup:]}
    server.completed = [r for r in server.completed if r.rid in keep]
    return server.stats()
