"""Helpers for the GPU parity tests: run the HIP path through the C ABI and unpack results."""
from __future__ import annotations

import numpy as np
import torch

from paper_2605_31419_amd import raster


def make(scene, intrs, poses, sigma=1.0, t_min=1e-6, fit=True, opacity_min=False, tight_tiles=False):
    sc = raster.DeviceScene.from_numpy(scene)
    rast = raster.Rasterizer(sc, intrs, raster.Params(sigma=sigma, t_min=t_min, opacity_min=opacity_min,
                                                      tight_tiles=tight_tiles))
    p = raster.poses_tensor(poses)
    if fit:
        rast.fit(p)
    return rast, p


def render(rast, p):
    rast.bin_and_sort(p)
    c, d, t = rast.forward(p)
    torch.cuda.synchronize()
    return c.cpu().numpy(), d.cpu().numpy(), t.cpu().numpy()


def per_view(rast, flat, ch):
    out, off = [], 0
    for it in rast.intrs:
        n = it.width * it.height
        out.append(flat[off * ch:(off + n) * ch].reshape(ch, n) if ch > 1 else flat[off:off + n])
        off += n
    return out


def binning_arrays(rast):
    """(K, pairs[K] sorted per tile, ranges[T, 2], tile_counts) copied to the host."""
    b = rast.binning()
    ws = rast.ws
    base = ws.data_ptr()

    def arr(ptr, n, dtype):
        off = ptr - base
        nbytes = n * np.dtype(dtype).itemsize
        return ws[off:off + nbytes].cpu().numpy().view(dtype)

    torch.cuda.synchronize()
    K = int(arr(b.n_pairs, 1, np.int64)[0])
    ranges = arr(b.ranges, 2 * b.n_tiles, np.uint32).reshape(-1, 2)
    pairs = arr(b.pairs, max(K, 0), np.uint64)
    counts = arr(b.tile_counts, rast.n_views * rast.scene.n_faces, np.uint32)
    overflow = int(arr(b.overflow, 1, np.uint32)[0])
    return K, pairs, ranges, counts, overflow


def to_dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32).reshape(-1), device="cuda")
