"""Writes the packaged tile-schedule table (``autotune_table.json``) by timing every candidate
schedule of the fused training kernel on the standard workloads, on the GPU it runs on:

    python -m paper_2605_31419_amd.tune_table [--out PATH] [--reps N]

Workloads: 64x48 with 2k faces, 640x480 with a 200k-face room soup (tracking step), the
8-view 1200x680 mapping window over a 500k-face room soup, one 1200x680 view of the 1M-face
mixed-size map, and 8 views of that map along a keyframe path.  Each entry is keyed by
(view sizes, number of views, log2 of the pair count) as ``autotune.lookup`` reads it.
"""
from __future__ import annotations

import argparse
import json

from . import autotune, raster, scenes


def _entry(dev, intrs, poses, target_poses, reps, table):
    import torch

    rast = raster.Rasterizer(dev, intrs)
    p = raster.poses_tensor(poses)
    tp = raster.poses_tensor(target_poses)
    k = rast.fit(p, slack=1.5)
    rast.ensure_capacity(int(max(k, rast.count(tp)) * 1.5) + 4096)
    rast.bin_and_sort(tp)
    tc, td, _ = rast.forward(tp)
    tc, td = tc.clone(), td.clone()
    best, times = autotune.tune(rast, p, tc, td, reps=reps)
    autotune.record(table, intrs, k, best, times)
    torch.cuda.synchronize()
    return autotune.key_for(intrs, k), best, times


def main(argv=None):
    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=autotune.DEFAULT_TABLE)
    ap.add_argument("--reps", type=int, default=7)
    args = ap.parse_args(argv)
    table = {}
    for name in ("single_64x48", "track_640x480", "window_8x1200x680", "track_1200x680_1M"):
        w = scenes.workload(name)
        dev = raster.DeviceScene.from_numpy(w.scene)
        key, best, times = _entry(dev, w.intr, w.poses, w.target_poses, args.reps, table)
        print(f"{name}: {key} -> {best}  {json.dumps({k: round(v, 4) for k, v in times.items()})}", flush=True)
        if name == "track_1200x680_1M":
            # a keyframe window of 8 views over the same map (the benchmark's batched path)
            g = scenes.rng(5500)
            poses = scenes.room_trajectory(g, 8)
            targets = [scenes.perturb_pose(p, g) for p in poses]
            key, best, times = _entry(dev, [w.intr[0]] * 8, poses, targets, args.reps, table)
            print(f"{name} x8: {key} -> {best}  {json.dumps({k: round(v, 4) for k, v in times.items()})}",
                  flush=True)
        del dev
        torch.cuda.empty_cache()
    autotune.save_table(table, args.out)
    print(f"wrote {len(table)} entries to {args.out}", flush=True)


if __name__ == "__main__":
    main()
