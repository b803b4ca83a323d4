#!/usr/bin/env python
"""Benchmark of the differentiable triangle-soup rasterizer on one MI355X.

One step = one pass of the whole hot path over one synthetic input: projection and setup,
tile binning and per-tile depth sort (tsr_bin_and_sort), then the fused forward render,
L1 colour + depth loss seeds and backward pass to vertex positions, colours, opacities and
the se(3) pose (tsr_render_train_l1).  Inputs are resident in HBM before timing starts.

Workload (default): a 1,000,000-face synthetic room soup (90 % of faces 0.5-2 cm, 10 %
5-20 cm), one 1200x680 view; targets rendered from the pose perturbed by 1 cm / 0.5 deg.
Also reported: the same step over a batch of 8 views of 1200x680 along a keyframe path,
the unfused path (forward, then backward from external seeds), per-kernel times (HIP events
on the launch stream), rooflines, and the FP64 oracle timed on the host cores.

Prints one JSON line.  --gpus N > 1 is not supported (one GPU per process, one GPU here).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_VECTOR_PEAK_TF = 157.3    # MI355X FP32 vector, published (packed); 78.6 without packed FP32
# FLOPs per (pixel, face) window evaluation (FMA = 2), counted from the inner loops of the
# blend kernels:
# forward 40 (offsets 2, 3 edge functions 12, min 2, alpha 1, colour planes 12, blend 11);
# backward 81 (re-evaluation 30, transmittance recovery 3, colour/depth weights and their
# x/y moments 11, dL/dalpha = T (P - S) 10, opacity/window 2, x/y moments of the edge that
# attains the minimum 2, update of S 3, summing the 20 per-pixel terms over the tile 20).
FLOP_FWD = 40
FLOP_BWD = 81


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--faces", type=int, default=1_000_000)
    ap.add_argument("--views", type=int, default=8, help="views of the batched measurement")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pixels", type=int, default=4096)
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="(kept for older profiler commands: the 256 MiB device copy now always runs)")
    ap.add_argument("--no-sigma-half", action="store_true", help="skip the headline step at the paper's sigma = 0.5")
    ap.add_argument("--tight-tiles", action="store_true",
                    help="bin with the tight triangle-tile test (same images and gradients, shorter lists)")
    ap.add_argument("--serve-warmup", type=int, default=500)
    ap.add_argument("--only-single", action="store_true", help="skip the unfused and batched legs")
    ap.add_argument("--only-window", action="store_true",
                    help="time only the 8-view mapping window (fused L1 step and the whole mapping energy)")
    ap.add_argument("--only-photometric", action="store_true",
                    help="after the headline step, time only the full photometric step (D-SSIM term)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile schedule (no autotuning)")
    ap.add_argument("--schedule", default=None,
                    help="fixed tile schedule 'persistent,order,grid' for the single view (no autotuning)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-track", action="store_true", help="skip the captured tracking-loop leg")
    ap.add_argument("--serve-queries", type=int, default=10000)
    ap.add_argument("--no-configs", action="store_true", help="skip the other configurations (64x48, 640x480, window)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Case:
    """A rasterizer with its inputs, outputs and gradient buffers resident on the device."""

    def __init__(self, raster, scenes, dev_scene, poses, intrs, target_poses, sigma=1.0, tight_tiles=False):
        import torch

        self.torch = torch
        self.rast = raster.Rasterizer(dev_scene, intrs, raster.Params(sigma=sigma, tight_tiles=tight_tiles))
        self.poses = raster.poses_tensor(poses)
        tposes = raster.poses_tensor(target_poses)
        self.K = self.rast.fit(self.poses, slack=1.5)
        Kt = self.rast.count(tposes)
        self.rast.ensure_capacity(int(max(self.K, Kt) * 1.5) + 4096)
        # targets: the same map rendered from the perturbed poses
        self.rast.bin_and_sort(tposes)
        tc, td, _ = self.rast.forward(tposes)
        self.tc, self.td = tc.clone(), td.clone()
        P = self.rast.total_pixels
        self.color = torch.empty(3 * P, device="cuda")
        self.depth = torch.empty(P, device="cuda")
        self.trans = torch.empty(P, device="cuda")
        self.loss = torch.empty(len(intrs), device="cuda")
        self.grads = self.rast.grad_buffers()
        self.pixels = P
        torch.cuda.synchronize()

    def step(self):
        self.rast.bin_and_sort(self.poses, check_capacity=False)
        self.rast.train_l1(self.poses, self.tc, self.td, color=self.color, depth=self.depth, trans=self.trans,
                           loss=self.loss, out=self.grads)

    def step_unfused(self, gc, gd):
        self.rast.bin_and_sort(self.poses, check_capacity=False)
        self.rast.forward(self.poses, self.color, self.depth, self.trans)
        self.rast.backward(self.poses, gc, gd, None, out=self.grads)

    def check(self):
        from paper_2605_31419_amd import _lib, raster

        _lib.check(self.rast.lib.tsr_check(raster._ptr(self.rast.ws), raster._stream(), None), "tsr_check")

    def evaluations(self):
        """Pixel-face window evaluations E of one pass, each pixel counting the faces of its
        tile's list up to its early stop (the whole list when it does not stop), plus the
        tile-list statistics, for the poses the step renders."""
        self.rast.bin_and_sort(self.poses)
        _, _, trans = self.rast.forward(self.poses)
        self.torch.cuda.synchronize()
        b = self.rast.binning()
        ws = self.rast.ws
        off = b.ranges - ws.data_ptr()
        rng = ws[off:off + 8 * b.n_tiles].cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
        lens = rng[:, 1] - rng[:, 0]
        loff = b.last_face - ws.data_ptr()
        last = ws[loff:loff + 4 * b.n_pixels].cpu().numpy().view(np.int32).astype(np.int64)
        T = trans.cpu().numpy()
        t_min = self.rast.params.t_min
        E = 0
        tile0 = pix0 = 0
        for it in self.rast.intrs:
            tx, ty = (it.width + 15) // 16, (it.height + 15) // 16
            ys, xs = np.mgrid[0:it.height, 0:it.width]
            t = (tile0 + (ys // 16) * tx + xs // 16).reshape(-1)
            P = it.width * it.height
            lp, Tp = last[pix0:pix0 + P], T[pix0:pix0 + P]
            stopped = (Tp < t_min) | (Tp == 0.0)
            E += int(np.where(stopped, lp - rng[t, 0] + 1, lens[t]).sum())
            tile0 += tx * ty
            pix0 += P
        kk = int(ws[b.n_pairs - ws.data_ptr():b.n_pairs - ws.data_ptr() + 8].cpu().numpy().view(np.int64)[0])
        cnt_off = b.tile_counts - ws.data_ptr()
        counts = ws[cnt_off:cnt_off + 4 * self.rast.n_views * self.rast.scene.n_faces].cpu().numpy().view(np.uint32)
        return E, kk, int((counts > 0).sum()), int(lens.max()), float(lens.mean())


def time_steps(fn, steps, warmup):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(steps):
        fn()
    b.record(st)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def step_stats(fn, steps, warmup):
    """Mean over `steps` back-to-back steps (events around the whole run, as the headline
    figure), plus the median, p99 and minimum of per-step times (an event between steps)."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(st)
    for i in range(steps):
        fn()
        ev[i + 1].record(st)
    torch.cuda.synchronize()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    return {"mean": ev[0].elapsed_time(ev[-1]) / steps, "median": float(np.median(per)),
            "p99": float(np.percentile(per, 99)), "min": float(per.min()), "steps": steps}


def graph_steps(case, steps, warmup):
    """The same step (binning + fused training) captured once in a HIP graph and replayed
    `steps` times back to back; returns (ms per step, largest relative norm deviation of the
    replayed gradients from an eager step's).  The step allocates nothing and clears its
    accumulators with kernels, so it replays as captured."""
    import torch

    case.step()
    torch.cuda.synchronize()
    ref = [x.clone() for x in case.grads]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            case.step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(steps):
        graph.replay()
    b.record(st)
    torch.cuda.synchronize()
    dev = max(float(torch.linalg.norm(x - r) / torch.linalg.norm(r).clamp_min(1e-30)) for x, r in zip(case.grads, ref))
    return a.elapsed_time(b) / steps, dev


def kernel_times(fn, steps):
    from paper_2605_31419_amd import _lib
    import torch

    torch.cuda.synchronize()
    _lib.profile_reset()
    _lib.profile_enable(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    prof = _lib.profile_read()
    _lib.profile_enable(False)
    _lib.profile_reset()
    return {k: v[1] / v[0] for k, v in prof.items()}, {k: v[0] // steps for k, v in prof.items()}


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed profiler-counter summary (FETCH_SIZE
    and WRITE_SIZE passes, scaled by a device copy of known size), or None when no summary
    covers this kernel or the sources changed since the counters were recorded."""
    import glob
    import re

    from paper_2605_31419_amd.build import source_fingerprint

    fp = source_fingerprint()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                m = re.match(r"\s*traffic: kernel=(\S+) fetch_bytes=(\d+) write_bytes=(\d+) sources=([0-9a-f]+)", line)
                if m and m.group(1).split("<")[0] == kernel and m.group(4) == fp:
                    return int(m.group(2)) + int(m.group(3)), os.path.relpath(path, ROOT)
    return None, None


# HBM bytes per colour value of the two D-SSIM kernels of the photometric step:
#   ssim_stats reads C and Cbar (8) and writes the maps A, B, C (12);
#   photo_seeds reads A, B, C (12), C and Cbar (8), writes dL/dC (4), and per pixel reads D and
#   Dbar and writes dL/dD (12 per pixel = 4 per colour value).
DSSIM_BYTES_PER_VALUE = 20 + 28
# The term itself needs at least C and Cbar once and dL/dC once: 12 bytes per colour value.
DSSIM_MIN_BYTES_PER_VALUE = 12


# E_equi reads the 9 coordinates of a soup face and writes their 9 gradients: 72 bytes per face.
EQUI_BYTES_PER_FACE = 72


def photometric_summary(pixels, ms, ktimes):
    dk = ("ssim_stats", "photo_seeds")
    d_ms = sum(ktimes.get(k, 0.0) for k in dk)
    values = 3 * pixels
    ach = DSSIM_BYTES_PER_VALUE * values / (d_ms * 1e-3) / 1e9
    return {"ms_per_step": ms, "mpix_s": pixels / (ms * 1e-3) / 1e6, "w_ssim": 0.2,
            "kernels_ms": {k: round(v, 4) for k, v in ktimes.items()},
            "dssim_roofline": {"kernels": list(dk), "bound": "hbm", "ms": d_ms, "achieved": ach,
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                               "algorithmic_bytes": DSSIM_BYTES_PER_VALUE * values,
                               "minimum_bytes_gbs": DSSIM_MIN_BYTES_PER_VALUE * values / (d_ms * 1e-3) / 1e9}}


def configs_leg(raster, scenes, steps, warmup):
    """The fused step on the other configurations: 64x48 with 2k faces, 640x480 with a 200k room
    soup (tracking step), and the 8-view 1200x680 mapping window over a 500k room soup."""
    import torch

    from paper_2605_31419_amd import autotune

    out = {}
    for name in ("single_64x48", "track_640x480", "window_8x1200x680"):
        w = scenes.workload(name)
        dev = raster.DeviceScene.from_numpy(w.scene)
        case = Case(raster, scenes, dev, w.poses, w.intr, w.target_poses)
        best, _ = autotune.tune(case.rast, case.poses, case.tc, case.td, reps=3)
        case.rast.schedule = best
        ms = time_steps(case.step, steps, warmup)
        case.check()
        out[name] = {"faces": int(w.scene.n_faces), "views": len(w.intr), "ms_per_step": ms,
                     "mpix_s": case.pixels / (ms * 1e-3) / 1e6, "schedule": list(best)}
        log(f"[bench] {name}: {ms:.3f} ms -> {out[name]['mpix_s']:.1f} Mpix/s")
        del case, dev
        torch.cuda.empty_cache()
    return out


def bin_sort_bytes(M, V, m_vis, K, n_tiles):
    """Algorithmic HBM bytes of projection + binning + sort with one sort pass (lower bound):
    positions 36 B/face, setup records 96 B per visible (view, face), counts 8 B per
    (view, face), emission 12 B per pair, one sort pass 24 B per pair, ranges 8 B per pair and
    8 B per tile."""
    return M * 36 + m_vis * 96 + V * M * 8 + K * 12 + K * 24 + K * 8 + n_tiles * 8


def tracking_leg(raster, w, dev, iters=100, schedule=None):
    """Tracking stress: `iters` pose-gradient iterations (bin, fused fwd+L1+bwd with pose
    gradient only, device pose step) captured once into a graph and replayed."""
    import torch

    from paper_2605_31419_amd.track import Tracker

    intr = w.intr[0]
    tr = raster.Rasterizer(dev, [intr])
    tp = raster.poses_tensor(w.target_poses)
    tr.fit(tp)
    tr.bin_and_sort(tp)
    tc, td, _ = tr.forward(tp)
    trk = Tracker(dev, intr, iters=iters, schedule=schedule)
    p0 = torch.as_tensor(w.poses[0], device="cuda")
    trk.set_frame(p0, tc, td)
    trk.capture()
    trk.set_frame(p0, tc, td)
    trk.replay()                                   # warm-up replay
    torch.cuda.synchronize()
    reps = 5
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    total = 0.0
    for _ in range(reps):
        trk.set_frame(p0, tc, td)
        a.record()
        trk.replay()
        b.record()
        torch.cuda.synchronize()
        total += a.elapsed_time(b)
    trk.check()
    lh = trk.loss_hist.cpu().numpy()
    eager = Tracker(dev, intr, iters=iters)
    eager.set_frame(p0, tc, td)
    torch.cuda.synchronize()
    a.record()
    eager.run_eager()
    b.record()
    torch.cuda.synchronize()
    ms_eager = a.elapsed_time(b)
    return {"iterations": iters, "ms_per_iteration": total / reps / iters,
            "ms_per_iteration_eager": ms_eager / iters, "loss_first": float(lh[0]), "loss_last": float(lh[-1])}


def serving_leg(raster, w, dev, n_queries, n_warm, seed=4400):
    """Continuous-batching render serving of the resident 1M-face map (forward colour + depth,
    resolutions uniform over 320x240 / 640x480 / 1200x680, random poses in the room):
    saturated throughput, then open-loop Poisson arrivals at 25 / 50 / 80 % of it, each over
    n_queries after n_warm warm-up queries, p50 / p99 latency per rate (8 GB budget, 4 slots,
    batches of up to 8 views).  The plain single-view path (one slot, one view per launch) is
    run at the same offered rates, and the batched server again under a tight 512 MB budget
    with one slot (a slot's workspace holds about 230 B per (view, face) besides its pairs, so
    two slots of a 1200x680 view of the 1M-face map do not fit in 512 MB).  Outputs are dropped
    at completion, so the budget bounds the server's memory."""
    from paper_2605_31419_amd import scenes
    from paper_2605_31419_amd.serve import GpuExecutor, Server, run_poisson

    ex = GpuExecutor(dev, pairs_per_tile=160.0)

    def run(qps, slots=4, views=8, budget=8 << 30, n=n_queries, warm=n_warm):
        srv = Server(ex, n_slots=slots, mem_budget=budget, max_batch_views=views, keep_outputs=False)
        srv.start()
        try:
            qs = scenes.serving_queries(seed + int(qps) % 1000, n + warm, qps=qps)
            st = run_poisson(srv, qs, warmup=warm)
        finally:
            srv.stop()
        st.update({"offered_qps": None if qps >= 1e6 else qps, "slots": slots, "budget_bytes": budget})
        return st

    run(1e7, n=40, warm=0)                               # warm-up: allocator, code objects
    sat = run(1e7)
    log(f"[bench] serving saturated: {sat['qps']:.0f} qps, p99 {sat['p99_ms']:.2f} ms")
    plain = run(1e7, slots=1, views=1)
    out = {"queries": n_queries, "warmup_queries": n_warm, "saturated": sat, "plain_single_view": plain,
           "rates": [], "plain_rates": []}
    for frac in (0.25, 0.5, 0.8):
        q = frac * sat["qps"]
        st = run(q)
        out["rates"].append(st)
        pl = run(q, slots=1, views=1)
        out["plain_rates"].append(pl)
        log(f"[bench] serving at {q:.0f} qps: p50 {st['p50_ms']:.2f} / p99 {st['p99_ms']:.2f} ms "
            f"(plain single view p50 {pl['p50_ms']:.2f} / p99 {pl['p99_ms']:.2f} ms)")
    try:
        tight_sat = run(1e7, slots=1, budget=512 << 20)
        tight_q = run(0.25 * tight_sat["qps"], slots=1, budget=512 << 20)
        out["tight_512MB"] = {"saturated": tight_sat, "at_25pct": tight_q}
        log(f"[bench] serving, 512 MB budget: {tight_sat['qps']:.0f} qps saturated, "
            f"p99 {tight_q['p99_ms']:.2f} ms at {tight_q['offered_qps']:.0f} qps")
    except ValueError as e:                              # budget too small for one slot
        out["tight_512MB"] = {"error": str(e)}
    out["capacity_retries"] = ex.retries
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _median_of_3(fn):
    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        fn()
        runs.append(time.perf_counter() - t0)
    return float(np.median(runs)), [round(r, 4) for r in runs]


def cpu_baseline(w, n_pix, seed=7):
    """The FP64 oracle on the host cores (median of 3 runs each): the headline frame's
    forward + backward on a seeded pixel sample at all threads and at one thread, the 64x48
    frame in full, a 640x480 forward sample, and the reference binner on the headline frame."""
    from oracle import oracle as O
    from paper_2605_31419_amd import scenes

    nproc = O.max_threads()
    intr = w.intr[0]
    g = np.random.default_rng(seed)
    pix = np.sort(g.choice(intr.width * intr.height, size=n_pix, replace=False)).astype(np.int64)
    n1 = max(64, n_pix // 16)
    pix1 = np.sort(g.choice(pix, size=n1, replace=False))

    def fwd_bwd(wl, pixels):
        it = wl.intr[0]
        n = it.width * it.height if pixels is None else pixels.size
        O.render(wl.scene, wl.poses[0], it, pixels=pixels)
        O.backward(wl.scene, wl.poses[0], it, np.full((3, n), 1.0 / (3 * it.width * it.height)),
                   np.full(n, 0.05 / (it.width * it.height)), None, pixels=pixels)

    O.set_threads(nproc)
    t_n, runs_n = _median_of_3(lambda: fwd_bwd(w, pix))
    O.set_threads(1)
    t_1, runs_1 = _median_of_3(lambda: fwd_bwd(w, pix1))
    O.set_threads(nproc)
    c1 = scenes.workload("single_64x48")
    c1_px = c1.intr[0].width * c1.intr[0].height
    t_c1, _ = _median_of_3(lambda: fwd_bwd(c1, None))
    O.set_threads(1)
    t_c1_1, _ = _median_of_3(lambda: fwd_bwd(c1, None))
    O.set_threads(nproc)
    c2 = scenes.workload("track_640x480")
    c2_pix = np.sort(g.choice(640 * 480, size=8192, replace=False)).astype(np.int64)
    t_c2, _ = _median_of_3(lambda: O.render(c2.scene, c2.poses[0], c2.intr[0], pixels=c2_pix))
    t_bin, _ = _median_of_3(lambda: O.bin_pairs(w.scene, w.poses, w.intr))
    return {"value": n_pix / t_n / 1e6, "unit": "Mpix/s", "cores": nproc, "kind": "oracle",
            "sample": f"{n_pix} seeded pixels of the 1200x680 view, forward + backward over all "
                      f"{w.scene.n_faces} faces, median of 3 runs ({t_n:.2f} s)",
            "cpu_model": _cpu_model(), "runs_s": runs_n,
            "single_thread": {"value": n1 / t_1 / 1e6, "unit": "Mpix/s", "pixels": n1, "runs_s": runs_1},
            "full_frame_extrapolated_s": {"threads_all": t_n * intr.width * intr.height / n_pix,
                                          "threads_1": t_1 * intr.width * intr.height / n1},
            "configs": {
                "single_64x48_fwd_bwd_full_frame": {"ms_all_threads": 1e3 * t_c1, "ms_1_thread": 1e3 * t_c1_1,
                                                    "mpix_s": c1_px / t_c1 / 1e6},
                "track_640x480_forward": {"pixels": 8192, "s": t_c2, "mpix_s": 8192 / t_c2 / 1e6,
                                          "full_frame_extrapolated_s": t_c2 * 640 * 480 / 8192},
                "reference_binner_1200x680_1M": {"s": t_bin, "note": "orc_bin: FP64 projection, pairs, std sort"}}}


def batched_leg(args, raster, scenes, dev, w):
    """The 8-view mapping window over the headline map: the fused L1 step over every (view, tile)
    (autotuned schedule) and the whole mapping energy (D-SSIM photometric and depth terms, E_equi
    and E_norm against the sensor normals of the target depth), with one binning and, for
    comparison, with the normal loss binned on its own."""
    import torch

    g = scenes.rng(5500)
    bposes = scenes.room_trajectory(g, args.views)
    btargets = [scenes.perturb_pose(p, g) for p in bposes]
    bcase = Case(raster, scenes, dev, bposes, [w.intr[0]] * args.views, btargets, tight_tiles=args.tight_tiles)
    Eb, Kb, mvb, maxb, meanb = bcase.evaluations()
    btuned = None
    if not args.no_tune:
        from paper_2605_31419_amd import autotune
        bbest, btimes = autotune.tune(bcase.rast, bcase.poses, bcase.tc, bcase.td, reps=3)
        bcase.rast.schedule = bbest
        btuned = {"schedule": list(bbest), "candidates_ms": {k: round(v, 4) for k, v in btimes.items()}}
        log(f"[bench] batched autotuned schedule {bbest}: {json.dumps(btuned['candidates_ms'])}")
    bst = step_stats(bcase.step, max(10, args.steps // 2), args.warmup)
    msb = bst["mean"]
    bcase.check()
    ktb, _ = kernel_times(bcase.step, max(2, args.profile_steps // 2))
    batched = {"n_views": args.views, "ms_per_step": msb, "step_stats_ms": bst,
               "mpix_s": bcase.pixels / (msb * 1e-3) / 1e6,
               "K": Kb, "visible": mvb, "max_list": maxb, "mean_list": meanb,
               "kernels_ms": {k: round(v, 4) for k, v in ktb.items()}, "schedule": btuned}
    log(f"[bench] batched {args.views} views: {msb:.3f} ms -> {batched['mpix_s']:.1f} Mpix/s")
    # the whole mapping energy over the same window: D-SSIM photometric term and depth L1,
    # E_equi and E_norm against the sensor normals of the target depth; one binning with the
    # normals as extra channels of the walks, and (for comparison) the normal loss as a
    # step of its own with a second binning
    from paper_2605_31419_amd.window import MappingWindow
    from paper_2605_31419_amd import _lib
    bintr = [w.intr[0]] * args.views
    tnorm = raster.sensor_normals(bcase.td, bintr)
    energy = {"weights": {"ssim": 0.2, "depth": 0.05, "equi": 1.2, "norm": 0.05}}
    for fused in (True, False):
        win = MappingWindow(dev, bintr, w_ssim=0.2, w_equi=1.2, w_norm=0.05, fused_mapping=fused)
        win.prepare(bcase.poses)
        map_step = lambda: win.step(bcase.poses, bcase.tc, bcase.td, target_normals=tnorm)
        msm = time_steps(map_step, max(5, args.steps // 4), args.warmup)
        _lib.check(win.rast.lib.tsr_check(raster._ptr(win.rast.ws), raster._stream(), None), "tsr_check")
        if fused:
            ktm, _ = kernel_times(map_step, max(2, args.profile_steps // 2))
            energy.update({"ms_per_step": msm, "mpix_s": bcase.pixels / (msm * 1e-3) / 1e6,
                           "kernels_ms": {k: round(v, 4) for k, v in ktm.items()}})
            log(f"[bench] mapping energy over {args.views} views, one binning: {msm:.3f} ms")
        else:
            energy["separate_normal_step_ms"] = msm
            log(f"[bench] mapping energy over {args.views} views, normal loss binned separately: {msm:.3f} ms")
        del win
    # the same step at the paper's rendering exponent (sigma = 0.5)
    win = MappingWindow(dev, bintr, raster.Params(sigma=0.5), w_ssim=0.2, w_equi=1.2, w_norm=0.05)
    win.prepare(bcase.poses)
    map_half = lambda: win.step(bcase.poses, bcase.tc, bcase.td, target_normals=tnorm)
    energy["sigma_0_5_ms_per_step"] = time_steps(map_half, max(5, args.steps // 4), args.warmup)
    _lib.check(win.rast.lib.tsr_check(raster._ptr(win.rast.ws), raster._stream(), None), "tsr_check")
    log(f"[bench] mapping energy over {args.views} views at sigma = 0.5: {energy['sigma_0_5_ms_per_step']:.3f} ms")
    del win
    batched["mapping_energy"] = energy
    del tnorm
    del bcase
    torch.cuda.empty_cache()
    return batched


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding of views "
              "is designed but not built", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2605_31419_amd import raster, scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log(f"[bench] generating the {args.faces}-face room soup")
    w = scenes.workload("track_1200x680_1M", n_faces=args.faces)
    dev = raster.DeviceScene.from_numpy(w.scene)
    if args.only_window:
        batched = batched_leg(args, raster, scenes, dev, w)
        print(json.dumps({"metric": f"mapping window: {args.views} views of 1200x680, fwd+bwd Mpix/s",
                          "value": batched["mpix_s"], "unit": "Mpix/s", "batched": batched}), flush=True)
        return
    single = Case(raster, scenes, dev, w.poses, w.intr, w.target_poses, tight_tiles=args.tight_tiles)
    E, K, m_vis, maxlen, meanlen = single.evaluations()
    log(f"[bench] single view: K={K} visible={m_vis} max list {maxlen} mean {meanlen:.1f} evals {E}")
    tuned = None
    if args.schedule:
        single.rast.schedule = tuple(int(x) for x in args.schedule.split(","))
        tuned = {"schedule": list(single.rast.schedule), "candidates_ms": None}
    elif not args.no_tune:
        from paper_2605_31419_amd import autotune
        best, times = autotune.tune(single.rast, single.poses, single.tc, single.td, reps=5)
        single.rast.schedule = best
        tuned = {"schedule": list(best), "candidates_ms": {k: round(v, 4) for k, v in times.items()}}
        log(f"[bench] autotuned schedule {best}: {json.dumps(tuned['candidates_ms'])}")
    head_stats = step_stats(single.step, args.steps, args.warmup)
    ms_eager = head_stats["mean"]
    single.check()
    log(f"[bench] fused step, eager launches: {ms_eager:.3f} ms -> {single.pixels / (ms_eager * 1e-3) / 1e6:.1f} Mpix/s")
    ms_graph, graph_dev = graph_steps(single, args.steps, args.warmup)
    single.check()
    log(f"[bench] fused step replayed from a HIP graph: {ms_graph:.3f} ms (gradients vs eager: {graph_dev:.1e} rel)")
    if graph_dev > 1e-4:
        raise RuntimeError(f"graph replay differs from the eager step ({graph_dev:.2e})")
    # the step is GPU-bound: replaying it from a graph gains nothing here (its node launches
    # cost more than the eager enqueue, which overlaps the kernels), so the eager time is quoted
    ms = ms_eager
    mpix = single.pixels / (ms * 1e-3) / 1e6
    log(f"[bench] fused step {ms:.3f} ms -> {mpix:.1f} Mpix/s")
    ktimes, klaunch = kernel_times(single.step, args.profile_steps)
    log(f"[bench] kernels (ms): {json.dumps({k: round(v, 4) for k, v in ktimes.items()})}")

    # measured device-copy bandwidth (also the calibration copy of the profiler-counter runs)
    n = 256 << 20
    src = torch.empty(n // 4, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(5):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * n * 5 / (a.elapsed_time(b) * 1e-3) / 1e9
    log(f"[bench] device copy of 256 MiB: {copy_gbs:.0f} GB/s (read + write)")
    del src, dst
    if args.only_single:
        print(json.dumps({"metric": "fwd+bwd Mpix/s (single view only)", "value": mpix, "unit": "Mpix/s",
                          "ms_per_step": ms, "kernels_ms": ktimes, "copy_gbs": copy_gbs, "schedule": tuned}), flush=True)
        return

    # full photometric step of eqs. 8 and 10: forward, L1 + D-SSIM + depth seeds, backward
    def step_photo():
        single.rast.bin_and_sort(single.poses, check_capacity=False)
        single.rast.train_photometric(single.poses, single.tc, single.td, w_ssim=0.2, color=single.color,
                                      depth=single.depth, trans=single.trans, loss=single.loss, out=single.grads)

    if args.only_photometric:
        msp = time_steps(step_photo, args.steps, args.warmup)
        single.check()
        ktp, _ = kernel_times(step_photo, args.profile_steps)
        print(json.dumps({"metric": "photometric step (L1 + D-SSIM + depth) Mpix/s, single view",
                          "value": single.pixels / (msp * 1e-3) / 1e6, "unit": "Mpix/s", "ms_per_step": msp,
                          "photometric": photometric_summary(single.pixels, msp, ktp)}), flush=True)
        return

    # unfused path (forward, then backward from external per-pixel seeds)
    gc = torch.full((3 * single.pixels,), 1e-6, device="cuda")
    gd = torch.full((single.pixels,), 1e-7, device="cuda")
    ms_unf = time_steps(lambda: single.step_unfused(gc, gd), args.steps, args.warmup)
    kt_unf, _ = kernel_times(lambda: single.step_unfused(gc, gd), args.profile_steps)

    ms_photo = time_steps(step_photo, args.steps, args.warmup)
    single.check()
    kt_photo, _ = kernel_times(step_photo, args.profile_steps)
    photometric = photometric_summary(single.pixels, ms_photo, kt_photo)
    log(f"[bench] photometric step (L1 + D-SSIM): {ms_photo:.3f} ms; D-SSIM kernels "
        f"{photometric['dssim_roofline']['ms'] * 1e3:.1f} us")

    # map-management kernels: E_equi over the whole map, per-face screen statistics of the view
    def step_equi():
        raster.equilateral(dev, weight=1.2, grad=eq_grad, loss=eq_loss)
    eq_grad = torch.empty(3, dev.n_vertices, device="cuda")
    eq_loss = torch.empty(1, device="cuda")
    ms_equi = time_steps(step_equi, args.steps, args.warmup)
    kt_equi, _ = kernel_times(step_equi, args.profile_steps)
    single.rast.bin_and_sort(single.poses)
    ms_stats = time_steps(lambda: single.rast.face_stats(single.poses), args.steps, args.warmup)
    kt_stats, _ = kernel_times(lambda: single.rast.face_stats(single.poses), args.profile_steps)
    eq_ms = kt_equi.get("equi", 0.0)
    eq_gbs = EQUI_BYTES_PER_FACE * dev.n_faces / (eq_ms * 1e-3) / 1e9 if eq_ms > 0 else None
    map_mgmt = {"equi_ms": ms_equi, "equi_kernels_ms": {k: round(v, 4) for k, v in kt_equi.items()},
                "equi_roofline": {"bound": "hbm", "achieved": eq_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": None if eq_gbs is None else eq_gbs / HBM_PEAK_GBS,
                                  "bytes_per_face": EQUI_BYTES_PER_FACE},
                "face_stats_ms": ms_stats, "face_stats_kernels_ms": {k: round(v, 4) for k, v in kt_stats.items()}}
    log(f"[bench] E_equi over {dev.n_faces} faces {ms_equi * 1e3:.1f} us; face statistics {ms_stats * 1e3:.1f} us")

    batched = None
    if not args.no_batched:
        batched = batched_leg(args, raster, scenes, dev, w)

    sigma_half = None
    if not args.no_sigma_half:
        # the headline step at the paper's rendering exponent (sigma = 0.5, square-root window)
        hcase = Case(raster, scenes, dev, w.poses, w.intr, w.target_poses, sigma=0.5, tight_tiles=args.tight_tiles)
        htuned = None
        if not args.no_tune:
            from paper_2605_31419_amd import autotune
            hbest, _ = autotune.tune(hcase.rast, hcase.poses, hcase.tc, hcase.td, reps=5)
            hcase.rast.schedule = hbest
            htuned = list(hbest)
        hst = step_stats(hcase.step, args.steps, args.warmup)
        hcase.check()
        sigma_half = {"sigma": 0.5, "ms_per_step": hst["mean"], "mpix_s": hcase.pixels / (hst["mean"] * 1e-3) / 1e6,
                      "step_stats_ms": hst, "schedule": htuned}
        log(f"[bench] sigma = 0.5: {hst['mean']:.3f} ms -> {sigma_half['mpix_s']:.1f} Mpix/s")
        del hcase

    tracking = None
    if not args.no_track:
        tracking = tracking_leg(raster, w, dev, schedule=single.rast.schedule)
        log(f"[bench] tracking graph: {tracking['ms_per_iteration']:.3f} ms/iteration over {tracking['iterations']}")
    serving = None
    if not args.no_serve:
        serving = serving_leg(raster, w, dev, args.serve_queries, args.serve_warmup)

    configs = None if args.no_configs else configs_leg(raster, scenes, args.steps, args.warmup)

    # rooflines
    bs_names = ["fill_tiles", "project", "scan_tiles", "emit", "tile_sort"]
    bs_ms = sum(ktimes.get(k, 0.0) for k in bs_names)
    n_tiles = single.rast.binning().n_tiles
    bs_bytes = bin_sort_bytes(args.faces, 1, m_vis, K, n_tiles)
    dom = max(ktimes, key=ktimes.get)
    if dom == "train_fused":
        flops = E * (FLOP_FWD + FLOP_BWD)
        ach = flops / (ktimes[dom] * 1e-3) / 1e12
        traffic, tsrc = counter_traffic("k_" + dom)
        roof = {"kernel": dom, "bound": "alu", "achieved": ach, "peak": FP32_VECTOR_PEAK_TF, "unit": "TFLOP/s",
                "frac": ach / FP32_VECTOR_PEAK_TF, "traffic": traffic,
                "work": f"{E} pixel-face evaluations x {FLOP_FWD + FLOP_BWD} FLOP"}
        if tsrc:
            roof["traffic_source"] = tsrc
    else:
        ach = bs_bytes / (bs_ms * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": None}
    bs_ach = bs_bytes / (bs_ms * 1e-3) / 1e9
    # measured HBM bytes of the binning kernels (profiler counters of this build), per step
    bs_traffic = 0
    for k in ("k_fill_u32", "k_project", "k_scan_tiles", "k_emit", "k_tile_sort"):
        tb, _ = counter_traffic(k)
        if tb is None:
            bs_traffic = None
            break
        bs_traffic += tb
    out = {
        "metric": "fwd+bwd Mpix/s at 1200x680, 1M tris (1 view vs batched); p50/p99 render latency",
        "value": mpix, "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "step_stats_ms": head_stats, "ms_per_step_graph": ms_graph, "graph_vs_eager_rel": graph_dev,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"1200x680 single view, {args.faces}-face synthetic room soup "
                               "(90% 0.5-2 cm, 10% 5-20 cm), binning + fused fwd + L1 + bwd incl. pose",
                   "faces": args.faces, "pairs": K, "visible_faces": m_vis},
        "roofline": roof,
        "bin_sort_roofline": {"bound": "hbm", "achieved": bs_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": bs_ach / HBM_PEAK_GBS, "ms": bs_ms, "algorithmic_bytes": bs_bytes,
                              "traffic": bs_traffic,
                              "traffic_gbs": None if bs_traffic is None else bs_traffic / (bs_ms * 1e-3) / 1e9},
        "kernels_ms": {k: round(v, 4) for k, v in ktimes.items()},
        "photometric": photometric,
        "map_management": map_mgmt,
        "unfused": {"ms_per_step": ms_unf, "mpix_s": single.pixels / (ms_unf * 1e-3) / 1e6,
                    "kernels_ms": {k: round(v, 4) for k, v in kt_unf.items()}},
        "batched": batched,
        "sigma_0_5": sigma_half,
        "schedule": tuned,
        "tracking": tracking,
        "serving": serving,
        "configs": configs,
        "copy_gbs": copy_gbs,
    }
    if not args.no_cpu_baseline:
        log(f"[bench] oracle on {args.cpu_pixels} pixels")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_pixels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
