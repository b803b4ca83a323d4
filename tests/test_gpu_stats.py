"""GPU parity of the per-face screen statistics (tsr_face_stats) against the FP64 reference:
areas within FP32 rounding of the FP64 setup, coverage inside the reference's certain/possible
interval per face, visibility between its certain and possible sets; at the 1200 x 680
1M-face size, properties that hold at any size plus the areas of sampled faces."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2605_31419_amd import raster
from paper_2605_31419_amd import scenes as S
from tests import gpu_util as G
from tests.helpers import IDENTITY, tiny_scene

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _gpu_stats(sc, intrs, poses, t_min=1e-6, sigma=1.0, opacity_min=False):
    rast, p = G.make(sc, intrs, poses, sigma=sigma, t_min=t_min, opacity_min=opacity_min)
    rast.bin_and_sort(p)
    area, cov, vis = rast.face_stats(p)
    torch.cuda.synchronize()
    return rast, p, area.cpu().numpy(), cov.cpu().numpy(), vis.cpu().numpy()


def _check_view(sc, pose, intr, area, cov, vis, t_min, sigma=1.0, opacity_min=False):
    a, lo, hi, vc, vp = O.face_stats(sc, pose, intr, t_min=t_min, sigma=sigma, opacity_min=opacity_min)
    assert np.all(np.abs(area - a) <= 1e-6 * np.maximum(a, 1.0)), np.abs(area - a).max()
    bad = np.nonzero((cov < lo) | (cov > hi))[0]
    assert bad.size == 0, [(int(m), int(lo[m]), int(cov[m]), int(hi[m])) for m in bad[:5]]
    v = vis.astype(bool)
    assert np.all(v[vc]) and not np.any(v & ~vp)
    _say(f"  faces {len(a)}: visible {int(v.sum())} (certain {int(vc.sum())}, possible {int(vp.sum())}), "
         f"covered pixels {int(cov.sum())}, ambiguous {int((hi - lo).sum())}")


@pytest.mark.parametrize("seed,t_min", [(11, 1e-6), (12, 0.3), (13, 0.9)])
def test_tiny_scenes(seed, t_min):
    sc, intr = tiny_scene(seed, n_faces=40, w=48, h=36, f=36.0)
    _, _, area, cov, vis = _gpu_stats(sc, [intr], [IDENTITY], t_min=t_min)
    _check_view(sc, IDENTITY, intr, area, cov, vis, t_min)


def test_room_5k_faces_ragged_160x118():
    sc = S.room_soup(21, 5000, size_range=(0.02, 0.2))
    g = S.rng(22)
    pose = S.random_room_pose(g)
    intr = S.intrinsics_for(160, 118)
    _, _, area, cov, vis = _gpu_stats(sc, [intr], [pose])
    _check_view(sc, pose, intr, area, cov, vis, 1e-6)


def test_views_are_packed_view_major():
    sc = S.room_soup(23, 3000, size_range=(0.02, 0.2))
    g = S.rng(24)
    poses = S.room_trajectory(g, 3)
    intrs = [S.intrinsics_for(96, 64), S.intrinsics_for(50, 37), S.intrinsics_for(64, 64)]
    _, _, area, cov, vis = _gpu_stats(sc, intrs, poses)
    M = sc.n_faces
    for v in range(3):
        _check_view(sc, poses[v], intrs[v], area[v * M:(v + 1) * M], cov[v * M:(v + 1) * M],
                    vis[v * M:(v + 1) * M], 1e-6)


def test_full_size_1200x680_1m_properties():
    w = S.workload("track_1200x680_1M")
    rast, p, area, cov, vis = _gpu_stats(w.scene, w.intr, w.poses)
    rast.forward(p)
    torch.cuda.synchronize()
    b = rast.binning()
    ws = rast.ws
    loff = b.last_face - ws.data_ptr()
    last = ws[loff:loff + 4 * b.n_pixels].cpu().numpy().view(np.int32)
    touched = int((last >= 0).sum())                 # pixels that blended a face
    off = b.tile_counts - ws.data_ptr()
    counts = ws[off:off + 4 * w.scene.n_faces].cpu().numpy().view(np.uint32)
    _say(f"  touched {touched}, sum coverage {int(cov.sum())}, visible {int(vis.sum())}, binned {int((counts > 0).sum())}")
    assert int(cov.sum()) == touched                 # every pixel that blends has one dominant face
    assert np.all(vis[cov > 0] == 1)                 # a dominant face is blended
    assert not np.any((vis == 1) & (counts == 0))    # only binned faces can be blended
    # areas of sampled faces against the reference run on those faces alone
    g = np.random.default_rng(0)
    ms = np.sort(g.choice(w.scene.n_faces, 4000, replace=False))
    idx = (3 * ms[:, None] + np.arange(3)).reshape(-1)
    sub = S.Scene(w.scene.pos[:, idx].copy(), w.scene.col[:, idx].copy(), w.scene.opa[idx].copy())
    ref = O.face_stats(sub, w.poses[0], w.intr[0])[0]
    got = area[ms]
    assert np.all(np.abs(got - ref) <= 1e-6 * np.maximum(ref, 1.0)), np.abs(got - ref).max()
    assert np.all((got > 0) == (counts[ms] > 0))     # the area is set exactly for the binned faces


def test_tile_lists_longer_than_the_visibility_bitmap():
    """5,000 faint faces stacked over one 16 x 16 tile: list positions past the kernel's
    4,096-bit visibility bitmap take the direct path; every face blends (T stays above t_min)."""
    g = np.random.default_rng(77)
    M = 5000
    z = g.uniform(1.0, 3.0, size=M)
    base = np.array([[-0.5, -0.45, 0.0], [0.55, -0.4, 0.0], [0.0, 0.6, 0.0]])    # covers the view centre
    pos = np.empty((3, 3 * M))
    for m in range(M):
        tri = (base + g.normal(scale=0.03, size=(3, 3))) * z[m] * 0.1
        tri[:, 2] = z[m]
        pos[:, 3 * m:3 * m + 3] = tri.T
    sc = S.Scene(pos.astype(np.float32), g.uniform(0, 1, size=(3, 3 * M)).astype(np.float32),
                 np.full(3 * M, 0.002, np.float32))
    intr = S.Intrinsics(16, 16, 40.0, 40.0, 7.5, 7.5)
    _, _, area, cov, vis = _gpu_stats(sc, [intr], [IDENTITY])
    _check_view(sc, IDENTITY, intr, area, cov, vis, 1e-6)
    assert vis.sum() > 4096


def test_minimum_opacity_rule():
    """Coverage and visibility follow the face opacity rule: with the minimum of the vertex
    opacities, alpha (and so every blending decision) changes."""
    sc, intr = tiny_scene(14, n_faces=40, w=48, h=36, f=36.0)
    g = np.random.default_rng(14)
    sc = S.Scene(sc.pos, sc.col, g.uniform(0.05, 1.0, size=sc.n_vertices).astype(np.float32))
    _, _, area, cov, vis = _gpu_stats(sc, [intr], [IDENTITY], t_min=0.3, opacity_min=True)
    _check_view(sc, IDENTITY, intr, area, cov, vis, 0.3, opacity_min=True)


@pytest.mark.parametrize("sigma", [0.5, 0.75, 1.5, 2.0])
def test_other_window_exponents(sigma):
    """Coverage and visibility at the paper's sigma = 0.5 and at exponents served by the
    generic-exponent kernels (0.75, 1.5)."""
    sc, intr = tiny_scene(15, n_faces=40, w=48, h=36, f=36.0)
    _, _, area, cov, vis = _gpu_stats(sc, [intr], [IDENTITY], t_min=0.3, sigma=sigma)
    _check_view(sc, IDENTITY, intr, area, cov, vis, 0.3, sigma=sigma)
