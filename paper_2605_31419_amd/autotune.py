"""Autotuner for the tile schedule of the fused training kernel.

The fused kernel (forward walk, L1 seeds, backward walk per tile; one wave per 8x8 quadrant)
can run one workgroup per tile in XCD-interleaved id order, one workgroup per tile in
longest-list-first order, or as persistent workgroups pulling tiles from a device queue in
either order, with a chosen number of workgroups.  Tile-list lengths vary by orders of magnitude (a face near the camera spans
hundreds of tiles), so the best schedule depends on the workload.  ``tune`` times every
candidate on the actual inputs (device events, median of repeats), checks that each candidate
reproduces the default's loss, and records the winner in a table keyed by
(view sizes, number of views, log2 of the pair count).  At run time ``lookup`` reads the
table (path from $TSR_AUTOTUNE_TABLE, else the packaged default) and never writes it.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "autotune_table.json")

Schedule = Tuple[int, int, int]          # (persistent, order, grid)

CANDIDATES: List[Schedule] = [
    (0, 0, 0), (0, 1, 0),
    (1, 0, 1024), (1, 0, 2048), (1, 0, 4096),
    (1, 1, 1024), (1, 1, 2048), (1, 1, 4096),
]


def table_path() -> str:
    return os.environ.get("TSR_AUTOTUNE_TABLE", DEFAULT_TABLE)


def key_for(intrs: Sequence, n_pairs: int) -> str:
    sizes = sorted({(int(i.width), int(i.height)) for i in intrs})
    kb = int(round(math.log2(max(n_pairs, 1))))
    return f"{'+'.join(f'{w}x{h}' for w, h in sizes)}|V={len(intrs)}|K=2^{kb}"


_cache: Dict[str, Dict] = {}


def load_table(path: Optional[str] = None) -> Dict:
    path = path or table_path()
    if path not in _cache:
        try:
            with open(path) as f:
                _cache[path] = json.load(f)
        except FileNotFoundError:
            _cache[path] = {}
    return _cache[path]


def lookup(intrs: Sequence, n_pairs: int, path: Optional[str] = None) -> Optional[Schedule]:
    """Schedule for this workload from the table (exact key, else the nearest pair-count bucket
    with the same view sizes and count), or None."""
    tab = load_table(path)
    k = key_for(intrs, n_pairs)
    if k in tab:
        return tuple(tab[k]["schedule"])
    prefix = k.rsplit("|", 1)[0]
    best = None
    kb = int(k.rsplit("2^", 1)[1])
    for key, val in tab.items():
        if key.startswith(prefix + "|"):
            d = abs(int(key.rsplit("2^", 1)[1]) - kb)
            if best is None or d < best[0]:
                best = (d, tuple(val["schedule"]))
    return None if best is None else best[1]


def tune(rast, poses, target_color, target_depth, reps: int = 5, candidates=CANDIDATES,
         verbose: bool = False) -> Tuple[Schedule, Dict[str, float]]:
    """Time each candidate schedule for this rasterizer / inputs; return (best, {name: ms})."""
    import torch

    rast.bin_and_sort(poses)
    n_pairs = rast.count(poses)
    loss = torch.zeros(rast.n_views, device="cuda")
    grads = rast.grad_buffers()
    times: Dict[str, float] = {}
    ref_loss = None
    for cand in candidates:
        run = lambda: rast.train_l1(poses, target_color, target_depth, loss=loss, out=grads, schedule=cand)
        run()
        torch.cuda.synchronize()
        lv = loss.detach().cpu().double()
        if ref_loss is None:
            ref_loss = lv
        elif not torch.allclose(lv, ref_loss, rtol=1e-5, atol=1e-9):
            raise RuntimeError(f"schedule {cand} changed the loss: {lv.tolist()} vs {ref_loss.tolist()}")
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            run()
            b.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        ms.sort()
        times[str(cand)] = ms[len(ms) // 2]
        if verbose:
            print(f"  schedule {cand}: {times[str(cand)]:.4f} ms", flush=True)
    best = min(candidates, key=lambda c: times[str(c)])
    return best, times


def record(table: Dict, intrs, n_pairs: int, best: Schedule, times: Dict[str, float]) -> None:
    table[key_for(intrs, n_pairs)] = {"schedule": list(best), "ms": times}


def save_table(table: Dict, path: Optional[str] = None) -> None:
    path = path or table_path()
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    _cache.pop(path, None)
