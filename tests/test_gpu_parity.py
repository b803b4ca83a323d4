"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: tile lists bit-exact (K, ranges, sorted (z key, face) pairs); images within 1e-4
absolute; gradients within 1e-3 relative (norm-wise, and element-wise with a floor of 1e-5
of the largest reference element).  Large workloads are checked on seeded pixel samples
and on the complete gradients of sampled faces.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2605_31419_amd import _lib, raster
from paper_2605_31419_amd import scenes as S
from tests import gpu_util as G
from tests.helpers import IDENTITY, grad_close, plain_scene, tiny_scene

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4


def _say(*a):
    print(*a, flush=True)


def _oracle_bins(scene, poses, intrs, sigma=1.0, tight=False):
    tile, zb, face, ranges = O.bin_pairs(scene, poses, intrs, sigma=sigma, tight_tiles=tight)
    return tile, zb, face, ranges


def _assert_bins_equal(rast, scene, poses, intrs, tight=False):
    K, pairs, ranges, counts, overflow = G.binning_arrays(rast)
    assert overflow == 0
    tile, zb, face, oranges = _oracle_bins(scene, poses, intrs, tight=tight)
    assert K == len(tile), (K, len(tile))
    assert np.array_equal(ranges.astype(np.int64), oranges), "tile ranges differ"
    got_z = (pairs >> np.uint64(32)).astype(np.uint32)
    got_f = (pairs & np.uint64(0xFFFFFFFF)).astype(np.int64)
    bad = np.nonzero((got_z != zb) | (got_f != face))[0]
    assert bad.size == 0, f"{bad.size} of {K} pairs differ, first at {bad[:5]}"
    return K


# ---------------------------------------------------------------------------- scenes

def _equal_depth_scene(n=300, seed=0):
    """Fronto-parallel faces all at z = 2 (every depth key equal: order by face id)."""
    g = np.random.default_rng(seed)
    xy = g.uniform(-0.8, 0.8, size=(n, 1, 2)) + g.uniform(-0.08, 0.08, size=(n, 3, 2))
    v = np.concatenate([xy, np.full((n, 3, 1), 2.0)], axis=2)
    return plain_scene(v, col=g.uniform(0, 1, (n, 3, 3)), opa=g.uniform(0.3, 1, (n, 3)))


def _huge_faces_scene(seed=0):
    """A few triangles close to the camera spanning the whole 640x480 frame (~1200 tiles)
    over a layer of small faces."""
    g = np.random.default_rng(seed)
    big = np.array([[[-3, -3, 0.5 + 0.1 * i], [3, -3, 0.6 + 0.1 * i], [0, 3, 0.55 + 0.1 * i]] for i in range(4)])
    small = S.frustum_soup(seed + 1, 2000, S.intrinsics_for(640, 480), size_range=(0.01, 0.05))
    sv = small.pos.T.reshape(-1, 3, 3)
    allv = np.concatenate([big, sv], axis=0)
    col = np.concatenate([g.uniform(0, 1, (4, 3, 3)), small.col.T.reshape(-1, 3, 3)])
    opa = np.concatenate([np.full((4, 3), 0.4), small.opa.reshape(-1, 3)])
    return plain_scene(allv, col=col, opa=opa)


def _long_tile_scene(n, seed=0, opa=(0.3, 1.0)):
    """n small faces inside one 16x16 tile (tile list longer than one LDS sort pass, and
    longer than the span of faces a blending workgroup stages at once)."""
    g = np.random.default_rng(seed)
    c = g.uniform(1, 15, size=(n, 1, 2)) + g.uniform(-1.5, 1.5, size=(n, 3, 2))
    z = g.uniform(1, 3, size=(n, 1, 1)) * np.ones((n, 3, 1))
    v = np.concatenate([(c - 7.5) * z / 20.0, z], axis=2)
    return plain_scene(v, col=g.uniform(0, 1, (n, 3, 3)), opa=g.uniform(*opa, (n, 3)))


def _pixel_scene(n, w, h, f=20.0, seed=0, size=3.0, opa=(0.3, 1.0)):
    """n small faces placed in pixel space over a w x h image (focal f, centred principal
    point), back-projected at depths 1-3."""
    g = np.random.default_rng(seed)
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    c = np.stack([g.uniform(0, w - 1, n), g.uniform(0, h - 1, n)], axis=1)[:, None, :]
    c = c + g.uniform(-size, size, size=(n, 3, 2))
    z = g.uniform(1, 3, size=(n, 1, 1)) * np.ones((n, 3, 1))
    xy = (c - np.array([cx, cy])) * z / f
    return plain_scene(np.concatenate([xy, z], axis=2), col=g.uniform(0, 1, (n, 3, 3)), opa=g.uniform(*opa, (n, 3)))


def _pixel_intr(w, h, f=20.0):
    return S.Intrinsics(w, h, f, f, (w - 1) / 2.0, (h - 1) / 2.0)


def _max_views_case():
    """TSR_MAX_VIEWS views of one map, sizes from 1x1 and single rows/columns to several
    ragged tiles, each camera looking at the same pixel-space soup from its own centre."""
    sizes = [(1, 1), (17, 1), (1, 17), (16, 16), (33, 9), (2, 2), (48, 31), (5, 64)] * (_lib.TSR_MAX_VIEWS // 8)
    assert len(sizes) == _lib.TSR_MAX_VIEWS
    return _pixel_scene(150, 40, 40, seed=11, size=4.0), [IDENTITY] * len(sizes), [_pixel_intr(w, h) for w, h in sizes]


def _offscreen_scene():
    g = np.random.default_rng(1)
    v = g.uniform(-1, 1, size=(50, 3, 3))
    v[..., 2] = -2.0                              # behind the camera
    return plain_scene(v)


def _boundary_scene(intr, pose, seed=0, z_near=0.1):
    """Faces placed on the culling boundaries, built in camera space and mapped to the world
    through a rotated pose (so the float32 world coordinates round differently from the
    camera-space ones): sub-pixel faces whose pixel range starts or ends within 1e-6..1e-3 px
    of a pixel centre, at the image borders and inside it, in u and in v; and faces whose
    nearest vertex sits within 1e-7..1e-4 relative of the near plane."""
    g = np.random.default_rng(seed)
    W, H = intr.width, intr.height
    tri = []
    deltas = [-1e-3, -1e-4, -1e-5, -1e-6, 0.0, 1e-6, 1e-5, 1e-4, 1e-3]
    cols = [0, 1, W // 2, W - 2, W - 1]
    rows = [0, 1, H // 2, H - 2, H - 1]
    for c in cols:
        for r in rows:
            for d in deltas:
                z = g.uniform(0.3, 4.0)
                # range starting just after (d > 0) or at/before (d <= 0) column c, then ending just before c
                tri.append(([c + d, r - 0.3], [c + 0.4, r], [c + d, r + 0.3], z))
                tri.append(([c - 0.4, r - 0.3], [c - d, r], [c - 0.4, r + 0.3], z))
                # the same in v
                tri.append(([c - 0.3, r + d], [c, r + 0.4], [c + 0.3, r + d], z))
                tri.append(([c - 0.3, r - 0.4], [c, r - d], [c + 0.3, r - 0.4], z))
    pts = []
    for a, b, c2, z in tri:
        pts.append([[(u - intr.cx) * z / intr.fx, (v - intr.cy) * z / intr.fy, z] for u, v in (a, b, c2)])
    for eps in [-1e-4, -1e-5, -1e-6, -1e-7, 1e-7, 1e-6, 1e-5, 1e-4]:
        for _ in range(12):
            zn = z_near * (1.0 + eps)
            u, v = g.uniform(10, W - 10), g.uniform(10, H - 10)
            q = np.array([[u, v], [u + 5, v + 1], [u + 2, v + 6]])
            zs = np.array([zn, zn * 1.02, zn * 1.05])
            pts.append([[(qq[0] - intr.cx) * zz / intr.fx, (qq[1] - intr.cy) * zz / intr.fy, zz] for qq, zz in zip(q, zs)])
    cam = np.array(pts, np.float64)                                   # [F, 3, 3] camera space
    R = pose[:9].astype(np.float64).reshape(3, 3)
    t = pose[9:].astype(np.float64)
    world = np.einsum("ji,fkj->fki", R, cam - t)                     # R^T (c - t)
    n = world.shape[0]
    return plain_scene(world, col=g.uniform(0, 1, (n, 3, 3)), opa=g.uniform(0.3, 1, (n, 3)))


def _boundary_case():
    intr = S.intrinsics_for(1200, 680)
    pose = S.look_pose([1.3, 0.7, 1.4], 0.7, 0.2)
    return _boundary_scene(intr, pose), [pose], [intr]


def _with_identity(sc, intr):
    return sc, [IDENTITY], [intr]


CASES = {
    "single_64x48": lambda: (S.workload("single_64x48").scene, [IDENTITY], [S.intrinsics_for(64, 48)]),
    "tiny_ragged_50x37": lambda: _with_identity(*tiny_scene(5, n_faces=60, w=50, h=37, f=40.0, size=(0.05, 1.0))),
    "equal_depth": lambda: (_equal_depth_scene(), [IDENTITY], [S.Intrinsics(64, 64, 40.0, 40.0, 31.5, 31.5)]),
    "huge_faces_640x480": lambda: (_huge_faces_scene(), [IDENTITY], [S.intrinsics_for(640, 480)]),
    "long_tile_800": lambda: (_long_tile_scene(1000, 5), [IDENTITY], [S.Intrinsics(16, 16, 20.0, 20.0, 7.5, 7.5)]),
    # faint faces: the walks reach the end of the 1000-face list (several staged spans)
    "long_tile_faint_1000": lambda: (_long_tile_scene(1000, 7, opa=(0.01, 0.05)), [IDENTITY],
                                     [S.Intrinsics(16, 16, 20.0, 20.0, 7.5, 7.5)]),
    "long_tile_5000": lambda: (_long_tile_scene(5000), [IDENTITY], [S.Intrinsics(16, 16, 20.0, 20.0, 7.5, 7.5)]),
    "long_tile_12000": lambda: (_long_tile_scene(12000, 3), [IDENTITY], [S.Intrinsics(16, 16, 20.0, 20.0, 7.5, 7.5)]),
    "offscreen": lambda: (_offscreen_scene(), [IDENTITY], [S.intrinsics_for(64, 48)]),
    "culling_boundaries_1200x680": _boundary_case,
    # boundary extremes: widest and tallest images (1024 tiles in one row / column), and the
    # maximum number of views with 1x1, single-row and single-column images among them
    "wide_16384x2": lambda: (_pixel_scene(400, 16384, 2, seed=3), [IDENTITY], [_pixel_intr(16384, 2)]),
    "tall_3x16384": lambda: (_pixel_scene(400, 3, 16384, seed=4), [IDENTITY], [_pixel_intr(3, 16384)]),
    "max_views_32": _max_views_case,
    "multi_view_mixed": lambda: (tiny_scene(7, n_faces=80, w=40, h=30)[0], [IDENTITY, IDENTITY, IDENTITY],
                                 [S.Intrinsics(40, 30, 30.0, 30.0, 19.5, 14.5), S.Intrinsics(33, 17, 25.0, 25.0, 16.0, 8.0),
                                  S.Intrinsics(64, 48, 45.0, 45.0, 31.5, 23.5)]),
}


def _case(name):
    sc, poses, intrs = CASES[name]()
    if not isinstance(poses, list):
        poses = [poses]
    if not isinstance(intrs, list):
        intrs = [intrs]
    return sc, poses, intrs


# ---------------------------------------------------------------------------- binning

@pytest.mark.parametrize("name", list(CASES))
def test_binning_bit_exact(name):
    _say(f"[binning] case={name}")
    sc, poses, intrs = _case(name)
    rast, p = G.make(sc, intrs, poses)
    rast.bin_and_sort(p)
    K = _assert_bins_equal(rast, sc, poses, intrs)
    _say(f"  K = {K}")


def _one_tile_scene(n, seed):
    """n faces each covering pixel centres of the single tile of a 16x16 view (so that the
    tile's list holds exactly n pairs), at depths drawn from 40 values (many equal keys, whose
    order is the face id)."""
    g = np.random.default_rng(seed)
    c = g.uniform(5.5, 9.5, size=(n, 1, 2))
    ang = g.uniform(0, 2 * np.pi, size=(n, 1)) + np.array([0.0, 2 * np.pi / 3, 4 * np.pi / 3])
    r = g.uniform(3.0, 4.0, size=(n, 3))
    px = c + np.stack([r * np.cos(ang), r * np.sin(ang)], axis=2)       # inradius >= 1.5 px
    z = (1.0 + 0.05 * g.integers(0, 40, size=(n, 1, 1))) * np.ones((n, 3, 1))
    v = np.concatenate([(px - 7.5) * z / 20.0, z], axis=2)
    return plain_scene(v, col=g.uniform(0, 1, (n, 3, 3)), opa=g.uniform(0.3, 1, (n, 3)))


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025,
                               4096, 4097])
def test_tile_sort_at_every_length_boundary(n):
    """One tile listing exactly n faces, at each boundary of the sort's paths (one-wave sorts
    of 1, 2, 4 and 8 keys per lane, the workgroup register sort up to 1,024 keys, the LDS sort
    up to 4,096, the merge beyond), with many equal depths: the list bit-exact against the
    oracle binner."""
    _say(f"[tile sort] one tile of {n} faces")
    sc = _one_tile_scene(n, seed=n)
    intrs = [S.Intrinsics(16, 16, 20.0, 20.0, 7.5, 7.5)]
    rast, p = G.make(sc, intrs, [IDENTITY])
    rast.bin_and_sort(p)
    assert _assert_bins_equal(rast, sc, [IDENTITY], intrs) == n


@pytest.mark.parametrize("name", list(CASES))
def test_tight_binning_bit_exact(name):
    """Tight triangle-tile lists against the oracle binner with the same FP64 rule."""
    _say(f"[tight binning] case={name}")
    sc, poses, intrs = _case(name)
    rast, p = G.make(sc, intrs, poses, tight_tiles=True)
    rast.bin_and_sort(p)
    K = _assert_bins_equal(rast, sc, poses, intrs, tight=True)
    K_loose = len(_oracle_bins(sc, poses, intrs)[0])
    _say(f"  K = {K} (bounding-box lists: {K_loose})")
    assert K <= K_loose


@pytest.mark.parametrize("name", ["single_64x48", "huge_faces_640x480", "multi_view_mixed", "long_tile_800",
                                  "culling_boundaries_1200x680", "max_views_32"])
def test_tight_binning_leaves_images_and_gradients_unchanged(name):
    """The pairs tight binning drops have alpha = 0 at every pixel of their tile, so the
    forward images are bitwise those of the bounding-box lists and the gradients equal up to
    the order of the floating-point atomics; the fused step's loss likewise."""
    sc, poses, intrs = _case(name)
    outs = []
    for tight in (False, True):
        rast, p = G.make(sc, intrs, poses, tight_tiles=tight)
        P = rast.total_pixels
        g = np.random.default_rng(5)
        gc, gd = G.to_dev(g.normal(size=3 * P)), G.to_dev(g.normal(size=P))
        tc, td = G.to_dev(g.uniform(0, 1, 3 * P)), G.to_dev(g.uniform(0.5, 4, P))
        rast.bin_and_sort(p)
        img = [x.cpu().numpy() for x in rast.forward(p)]
        grads = [x.cpu().numpy() for x in rast.backward(p, gc, gd, None)]
        loss = torch.zeros(len(poses), device="cuda")
        fused = [x.cpu().numpy() for x in rast.train_l1(p, tc, td, loss=loss)]
        torch.cuda.synchronize()
        outs.append((img, grads, fused, loss.cpu().numpy()))
    for a, b in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, b)
    for a, b in zip(outs[0][1] + outs[0][2], outs[1][1] + outs[1][2]):
        np.testing.assert_allclose(b, a, rtol=1e-5, atol=1e-6 * max(np.abs(a).max(), 1e-30))
    np.testing.assert_allclose(outs[1][3], outs[0][3], rtol=1e-6)


def test_empty_scene_bins_nothing():
    sc = S.Scene(np.zeros((3, 0), np.float32), np.zeros((3, 0), np.float32), np.zeros(0, np.float32))
    rast, p = G.make(sc, [S.intrinsics_for(64, 48)], [IDENTITY], fit=False)
    rast.bin_and_sort(p)
    c, d, t = rast.forward(p)
    torch.cuda.synchronize()
    assert np.all(c.cpu().numpy() == 0) and np.all(d.cpu().numpy() == 0) and np.all(t.cpu().numpy() == 1)


def test_capacity_overflow_is_reported_and_harmless():
    w = S.workload("single_64x48")
    rast, p = G.make(w.scene, w.intr, w.poses, fit=False)
    rast.ensure_capacity(10)
    from paper_2605_31419_amd import _lib
    lib = _lib.load()
    import ctypes as C
    _lib.check(lib.tsr_bin_and_sort(*rast._args(p), raster._stream()), "bin")
    k = C.c_int64(0)
    rc = lib.tsr_check(raster._ptr(rast.ws), raster._stream(), C.byref(k))
    assert rc == _lib.TSR_ECAPACITY and k.value > 10
    c, d, t = rast.forward(p)                     # empty tile lists: background only
    torch.cuda.synchronize()
    assert np.all(t.cpu().numpy() == 1)
    rast.bin_and_sort(p)                          # grows and re-bins
    assert rast.capacity >= k.value


# ---------------------------------------------------------------------------- forward

FWD_CASES = ["single_64x48", "tiny_ragged_50x37", "equal_depth", "huge_faces_640x480", "long_tile_800",
             "long_tile_faint_1000", "long_tile_5000", "multi_view_mixed", "wide_16384x2", "tall_3x16384",
             "max_views_32"]


@pytest.mark.parametrize("name", FWD_CASES)
@pytest.mark.parametrize("sigma", [1.0, 0.5, 2.0, 0.75, 1.5])
def test_forward_matches_oracle(name, sigma):
    _say(f"[forward] case={name} sigma={sigma}")
    sc, poses, intrs = _case(name)
    rast, p = G.make(sc, intrs, poses, sigma=sigma)
    c, d, t = G.render(rast, p)
    cs, ds, ts = G.per_view(rast, c, 3), G.per_view(rast, d, 1), G.per_view(rast, t, 1)
    for v in range(len(poses)):
        oc, od, ot = O.render(sc, poses[v], intrs[v], sigma=sigma)
        err = max(np.abs(cs[v] - oc).max(), np.abs(ds[v] - od).max(), np.abs(ts[v] - ot).max())
        _say(f"  view {v}: max abs err {err:.3e}, covered px {(ot < 1).sum()}")
        assert err <= IMG_TOL


def test_forward_is_deterministic():
    w = S.workload("single_64x48")
    rast, p = G.make(w.scene, w.intr, w.poses)
    ref = G.render(rast, p)
    for _ in range(5):
        out = G.render(rast, p)
        for a, b in zip(ref, out):
            assert np.array_equal(a, b)


# ---------------------------------------------------------------------------- backward

BWD_CASES = ["single_64x48", "tiny_ragged_50x37", "equal_depth", "multi_view_mixed", "huge_faces_640x480",
             "long_tile_800", "long_tile_faint_1000", "wide_16384x2", "tall_3x16384", "max_views_32"]


def _gpu_backward(rast, p, gc, gd, gt):
    rast.bin_and_sort(p)
    rast.forward(p)
    out = rast.backward(p, G.to_dev(gc), G.to_dev(gd), None if gt is None else G.to_dev(gt))
    torch.cuda.synchronize()
    return [x.cpu().numpy().astype(np.float64) for x in out]


def _oracle_backward_views(sc, poses, intrs, gcs, gds, gts, sigma, with_abs=False):
    acc = None
    absacc = None
    gposes = []
    for v in range(len(poses)):
        out = O.backward(sc, poses[v], intrs[v], gcs[v], gds[v], None if gts is None else gts[v], sigma=sigma,
                         with_abs=with_abs)
        gp, gc, go, gpose = out[:4]
        acc = [gp, gc, go] if acc is None else [a + b for a, b in zip(acc, [gp, gc, go])]
        if with_abs:
            absacc = list(out[4]) if absacc is None else [a + b for a, b in zip(absacc, out[4])]
        gposes.append(gpose)
    res = acc + [np.concatenate(gposes)]
    return (res, absacc) if with_abs else res


# Pixels whose per-pixel gradient terms an FP32 implementation cannot reproduce to the relative
# bar, found from the oracle's discrete state (the rejection rule for ridge, edge and steep-slope
# flips), get zero upstream gradients on both sides (the same seeds go to the GPU and to the
# oracle); every other pixel is compared element-wise:
#  * steep-edge band (sigma < 1): the window's slope sigma rho^(sigma-1) grows without bound as
#    rho -> 0+, so within |rho| < 1e-3 of any face's edge the kernels' rounding of rho (a few
#    1e-7) changes per-pixel terms by more than the bar, and a face can be blended on one side
#    and not on the other;
#  * ridges of phi: where a blended face's two smallest normalised edge distances are within
#    1e-5 of each other (about 30 times the FP32 rounding of E_k), which edge attains the
#    minimum -- and so which edge's parameters receive that pixel's window gradient -- can flip.
STEEP_RHO = 1e-3
RIDGE_GAP = 1e-5


def _steep_masks(sc, poses, intrs, sigma):
    out = []
    for v in range(len(poses)):
        m = O.ridge_gap(sc, poses[v], intrs[v], sigma=sigma) < RIDGE_GAP
        if sigma < 1.0:
            m |= O.min_rho(sc, poses[v], intrs[v], sigma=sigma) < STEEP_RHO
        out.append(m)
    return out


def _apply_masks(flat, masks, ch):
    """Zero a packed per-view seed array at the masked pixels (in place)."""
    off = 0
    for m in masks:
        n = m.size
        seg = flat[off * ch:(off + n) * ch].reshape(ch, n) if ch > 1 else flat[off:off + n]
        seg[..., m] = 0.0
        off += n


@pytest.mark.parametrize("name", BWD_CASES)
@pytest.mark.parametrize("sigma", [1.0, 0.5, 2.0, 0.75, 1.5])
def test_backward_matches_oracle(name, sigma):
    _say(f"[backward] case={name} sigma={sigma}")
    sc, poses, intrs = _case(name)
    rast, p = G.make(sc, intrs, poses, sigma=sigma)
    P = rast.total_pixels
    g = np.random.default_rng(42)
    gc = g.normal(size=3 * P).astype(np.float32)
    gd = g.normal(size=P).astype(np.float32)
    gt = g.normal(size=P).astype(np.float32)
    masks = _steep_masks(sc, poses, intrs, sigma)
    for a, ch in ((gc, 3), (gd, 1), (gt, 1)):
        _apply_masks(a, masks, ch)
    _say(f"  steep-edge and ridge pixels masked on both sides: {sum(int(m.sum()) for m in masks)} of {P}")
    got = _gpu_backward(rast, p, gc, gd, gt)
    gcs = G.per_view(rast, gc, 3)
    gds, gts = G.per_view(rast, gd, 1), G.per_view(rast, gt, 1)
    ref, conds = _oracle_backward_views(sc, poses, intrs, gcs, gds, gts, sigma, with_abs=True)
    for nm, a, b, cond in zip(["grad_pos", "grad_col", "grad_opa", "grad_pose"], got, ref, conds + [None]):
        ok, msg, bad = grad_close(a, b, name=nm, cond=cond)
        _say("  " + msg)
        assert ok, msg


# ---------------------------------------------------------------------------- fused L1 step

def _nudged_targets(oc, od, seed, shape_hw):
    """Random colour/depth targets pushed at least 1e-3 away from the oracle render, so the
    sign of each L1 residual is the same in FP32 and FP64."""
    g = np.random.default_rng(seed)
    tc = g.uniform(0, 1, size=oc.shape)
    td = g.uniform(0.5, 4.0, size=od.shape)
    near_c = np.abs(tc - oc) < 1e-3
    tc[near_c] = oc[near_c] + 2e-3
    near_d = np.abs(td - od) < 1e-3
    td[near_d] = od[near_d] + 2e-3
    return tc.astype(np.float32), td.astype(np.float32), int(near_c.sum() + near_d.sum())


@pytest.mark.parametrize("name,sigma", [("single_64x48", 1.0), ("multi_view_mixed", 1.0), ("tiny_ragged_50x37", 1.0),
                                        ("long_tile_800", 1.0), ("long_tile_faint_1000", 1.0), ("max_views_32", 1.0),
                                        ("single_64x48", 2.0), ("multi_view_mixed", 1.5), ("tiny_ragged_50x37", 1.5)])
def test_train_l1_matches_oracle(name, sigma):
    _say(f"[train_l1] case={name} sigma={sigma}")
    sc, poses, intrs = _case(name)
    rast, p = G.make(sc, intrs, poses, sigma=sigma)
    tcs, tds, ocs, ods, lossref, gseeds = [], [], [], [], [], []
    for v in range(len(poses)):
        oc, od, ot = O.render(sc, poses[v], intrs[v], sigma=sigma)
        tc, td, nudged = _nudged_targets(oc, od, 100 + v, None)
        tcs.append(tc); tds.append(td)
        L, gcv, gdv = O.l1_seeds(oc, od, tc, td, intrs[v].width * intrs[v].height)
        lossref.append(L)
        gseeds.append((gcv, gdv))
        _say(f"  view {v}: nudged {nudged} targets")
    rast.bin_and_sort(p)
    P = rast.total_pixels
    loss = torch.zeros(len(poses), device="cuda")
    color = torch.empty(3 * P, device="cuda")
    depth = torch.empty(P, device="cuda")
    out = rast.train_l1(p, G.to_dev(np.concatenate([t.reshape(-1) for t in tcs])),
                        G.to_dev(np.concatenate([t.reshape(-1) for t in tds])), color=color, depth=depth, loss=loss)
    torch.cuda.synchronize()
    got = [x.cpu().numpy().astype(np.float64) for x in out]
    np.testing.assert_allclose(loss.cpu().numpy(), lossref, rtol=1e-5)
    ref = _oracle_backward_views(sc, poses, intrs, [s[0] for s in gseeds], [s[1] for s in gseeds], None, sigma)
    for nm, a, b in zip(["grad_pos", "grad_col", "grad_opa", "grad_pose"], got, ref):
        ok, msg, bad = grad_close(a, b, name=nm)
        _say("  " + msg)
        assert ok, msg
    cs = G.per_view(rast, color.cpu().numpy(), 3)
    for v in range(len(poses)):
        oc, od, ot = O.render(sc, poses[v], intrs[v], sigma=sigma)
        assert np.abs(cs[v] - oc).max() <= IMG_TOL


# ---------------------------------------------------------------------------- full photometric step

@pytest.mark.parametrize("name,sigma", [("single_64x48", 1.0), ("multi_view_mixed", 1.0), ("tiny_ragged_50x37", 1.0),
                                        ("long_tile_800", 1.0), ("single_64x48", 0.5), ("tiny_ragged_50x37", 2.0),
                                        ("tiny_ragged_50x37", 0.75), ("multi_view_mixed", 1.5)])
def test_train_photometric_matches_oracle(name, sigma):
    """Eqs. 8 and 10 with the D-SSIM term: the seeds are the oracle's L1 seeds plus 0.2 times
    the FP64 D-SSIM gradient of the oracle render, pushed through the oracle backward."""
    from oracle import dssim as D
    _say(f"[train_photometric] case={name} sigma={sigma}")
    w_ssim = 0.2
    sc, poses, intrs = _case(name)
    rast, p = G.make(sc, intrs, poses, sigma=sigma)
    tcs, tds, lossref, gcs, gds, ocs = [], [], [], [], [], []
    for v in range(len(poses)):
        W, H = intrs[v].width, intrs[v].height
        oc, od, ot = O.render(sc, poses[v], intrs[v], sigma=sigma)
        tc, td, _ = _nudged_targets(oc, od, 300 + v, None)
        L, gcv, gdv = O.l1_seeds(oc, od, tc, td, W * H)
        c3, t3 = np.asarray(oc, np.float64).reshape(3, H, W), tc.astype(np.float64).reshape(3, H, W)
        lossref.append(L + w_ssim * D.dssim(c3, t3))
        gcs.append(gcv + w_ssim * D.dssim_grad(c3, t3).reshape(gcv.shape))
        gds.append(gdv)
        tcs.append(tc); tds.append(td); ocs.append(oc)
    rast.bin_and_sort(p)
    P = rast.total_pixels
    loss = torch.zeros(len(poses), device="cuda")
    color = torch.empty(3 * P, device="cuda")
    depth = torch.empty(P, device="cuda")
    out = rast.train_photometric(p, G.to_dev(np.concatenate([t.reshape(-1) for t in tcs])),
                                 G.to_dev(np.concatenate([t.reshape(-1) for t in tds])), w_ssim=w_ssim,
                                 color=color, depth=depth, loss=loss)
    torch.cuda.synchronize()
    got = [x.cpu().numpy().astype(np.float64) for x in out]
    _say(f"  loss {loss.cpu().numpy()} ref {np.array(lossref)}")
    np.testing.assert_allclose(loss.cpu().numpy(), lossref, rtol=1e-5, atol=2e-5)
    ref, conds = _oracle_backward_views(sc, poses, intrs, gcs, gds, None, sigma, with_abs=True)
    for nm, a, b, cond in zip(["grad_pos", "grad_col", "grad_opa", "grad_pose"], got, ref, conds + [None]):
        ok, msg, bad = grad_close(a, b, name=nm, cond=cond)
        _say("  " + msg)
        assert ok, msg
    cs = G.per_view(rast, color.cpu().numpy(), 3)
    for v in range(len(poses)):
        assert np.abs(cs[v] - ocs[v]).max() <= IMG_TOL


# ---------------------------------------------------------------------------- minimum opacity rule

@pytest.mark.parametrize("name", ["single_64x48", "multi_view_mixed", "tiny_ragged_50x37"])
def test_minimum_opacity_rule_matches_oracle(name):
    """Face opacity = min of the vertex opacities: forward and backward against the oracle
    with the same rule; opacity gradients land on one vertex per face."""
    _say(f"[opacity_min] case={name}")
    sc, poses, intrs = _case(name)
    g = np.random.default_rng(9)
    sc = S.Scene(sc.pos, sc.col, g.uniform(0.2, 0.95, size=sc.n_vertices).astype(np.float32), sc.faces)
    rast, p = G.make(sc, intrs, poses, opacity_min=True)
    c, d, t = G.render(rast, p)
    cs, ds = G.per_view(rast, c, 3), G.per_view(rast, d, 1)
    for v in range(len(poses)):
        oc, od, ot = O.render(sc, poses[v], intrs[v], opacity_min=True)
        err = max(np.abs(cs[v] - oc).max(), np.abs(ds[v] - od).max())
        assert err <= IMG_TOL, (v, err)
    P = rast.total_pixels
    gc = g.normal(size=3 * P).astype(np.float32)
    gd = g.normal(size=P).astype(np.float32)
    got = _gpu_backward(rast, p, gc, gd, None)
    acc = None
    gposes = []
    for v, (gcv, gdv) in enumerate(zip(G.per_view(rast, gc, 3), G.per_view(rast, gd, 1))):
        out = O.backward(sc, poses[v], intrs[v], gcv, gdv, None, opacity_min=True)
        acc = list(out[:3]) if acc is None else [a + b for a, b in zip(acc, out[:3])]
        gposes.append(out[3])
    ref = acc + [np.concatenate(gposes)]
    for nm, a, b in zip(["grad_pos", "grad_col", "grad_opa", "grad_pose"], got, ref):
        ok, msg, _ = grad_close(a, b, name=nm)
        _say("  " + msg)
        assert ok, msg
    go = np.asarray(got[2]).reshape(-1)
    if sc.faces is None:
        per_face = (go.reshape(-1, 3) != 0).sum(axis=1)
        assert per_face.max() <= 1


# ---------------------------------------------------------------------------- pose step

def test_pose_step_matches_matrix_exponential():
    from tests.helpers import left_perturb
    g = np.random.default_rng(5)
    poses = np.stack([left_perturb(IDENTITY, g.normal(scale=0.3, size=6)) for _ in range(3)]).astype(np.float32)
    grad = g.normal(size=(3, 6)).astype(np.float32)
    pt = torch.as_tensor(poses.copy(), device="cuda").reshape(-1).contiguous()
    gt = torch.as_tensor(grad, device="cuda").reshape(-1).contiguous()
    from paper_2605_31419_amd import _lib
    lib = _lib.load()
    _lib.check(lib.tsr_pose_step(raster._ptr(pt), raster._ptr(gt), 3, 0.01, 0.02, raster._stream()), "pose_step")
    torch.cuda.synchronize()
    out = pt.cpu().numpy().reshape(3, 12)
    for v in range(3):
        tau = -np.concatenate([0.01 * grad[v, :3], 0.02 * grad[v, 3:]]).astype(np.float64)
        ref = left_perturb(poses[v].astype(np.float64), tau)
        np.testing.assert_allclose(out[v], ref, atol=2e-6)


# ---------------------------------------------------------------------------- output overwrite

@pytest.mark.parametrize("name", ["single_64x48", "multi_view_mixed"])
@pytest.mark.parametrize("fused", [False, True], ids=["separate", "fused"])
def test_gradients_overwrite_their_outputs(name, fused):
    """Gradient outputs are overwritten, whatever they held: with NaN-filled buffers the results
    equal those written into fresh buffers, and the vertices of faces no view sees come back
    exactly 0 (the vertex gather writes every vertex of a soup)."""
    _say(f"[overwrite] case={name} fused={fused}")
    sc, poses, intrs = _case(name)
    rast, p = G.make(sc, intrs, poses)
    rast.bin_and_sort(p)
    P = rast.total_pixels
    g = np.random.default_rng(7)
    if fused:
        c, d, _ = rast.forward(p)
        tc = G.to_dev(g.uniform(0, 1, 3 * P).astype(np.float32))
        td = G.to_dev(g.uniform(0.5, 4, P).astype(np.float32))
        run = lambda out: rast.train_l1(p, tc, td, out=out)
    else:
        rast.forward(p)
        gc = G.to_dev(g.normal(size=3 * P).astype(np.float32))
        gd = G.to_dev(g.normal(size=P).astype(np.float32))
        run = lambda out: rast.backward(p, gc, gd, None, out=out)
    ref = [x.clone() for x in run(None)]
    bufs = [torch.full_like(x, float("nan")) for x in ref]
    got = run(bufs)
    torch.cuda.synchronize()
    seen = np.zeros(sc.n_faces, bool)
    for v in range(len(poses)):
        _, _, _, tiles = O.project(sc, poses[v], intrs[v])
        seen |= tiles > 0
    unseen_v = np.repeat(~seen, 3)
    assert unseen_v.any() and seen.any()
    for nm, a, b in zip(["pos", "col", "opa", "pose"], got, ref):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.isfinite(a).all(), nm
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-9, err_msg=nm)
        if nm != "pose":
            per_vertex = a.reshape(-1, sc.n_vertices)
            assert (per_vertex[:, unseen_v] == 0).all(), nm


def test_last_face_positions_are_in_their_tiles():
    """The binning view's per-pixel last blended face: -1 only where nothing was blended (final
    transmittance 1, and every pixel with transmittance below 1 has one), otherwise a position
    inside the pixel's tile range whose face covers the pixel (oracle: that face alone gives
    the pixel a nonzero alpha)."""
    sc, poses, intrs = _case("tiny_ragged_50x37")
    rast, p = G.make(sc, intrs, poses)
    rast.bin_and_sort(p)
    _, _, trans = rast.forward(p)
    torch.cuda.synchronize()
    b = rast.binning()
    ws = rast.ws
    last = ws[b.last_face - ws.data_ptr():b.last_face - ws.data_ptr() + 4 * b.n_pixels].cpu().numpy().view(np.int32)
    rng = ws[b.ranges - ws.data_ptr():b.ranges - ws.data_ptr() + 8 * b.n_tiles].cpu().numpy().view(np.uint32)
    rng = rng.reshape(-1, 2).astype(np.int64)
    pairs = ws[b.pairs - ws.data_ptr():b.pairs - ws.data_ptr() + 8 * b.capacity].cpu().numpy().view(np.uint64)
    T = trans.cpu().numpy()
    it = intrs[0]
    tx = (it.width + 15) // 16
    ys, xs = np.mgrid[0:it.height, 0:it.width]
    t = ((ys // 16) * tx + xs // 16).reshape(-1)
    none = last < 0
    assert (T[none] == 1.0).all() and not none[T < 1.0].any()
    assert ((last[~none] >= rng[t[~none], 0]) & (last[~none] < rng[t[~none], 1])).all()
    faces = (pairs[last[~none]] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    pix = np.nonzero(~none)[0]
    for f, q in list(zip(faces, pix))[::7]:
        one = plain_scene(sc.pos.T.reshape(-1, 3, 3)[f:f + 1], col=sc.col.T.reshape(-1, 3, 3)[f:f + 1],
                          opa=sc.opa.reshape(-1, 3)[f:f + 1])
        _, _, ot = O.render(one, poses[0], it, pixels=np.array([q], np.int64))
        assert ot[0] < 1.0, (f, q)
