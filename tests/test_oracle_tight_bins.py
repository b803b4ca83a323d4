"""Pins of the oracle's tight triangle-tile binning (a binning variant outside the paper: a
face is listed only in the tiles of its pixel rectangle whose box of pixel centres can hold a
pixel it covers, i.e. where every edge function of eq. 2 reaches below 0).

* closed forms: the right triangle (0,0), (63,0), (0,63) at unit depth and focal length spans
  4 x 4 tiles; its hypotenuse u + v = 63 leaves the tiles with x + y <= 3 -- 10 of 16.  The
  triangle (8,8), (32,8), (8,32) spans 3 x 3 tiles; with each tile's box clipped to the pixel
  rectangle [8, 32]^2 the hypotenuse u + v = 40 reaches 0 at best in tiles (2,0) and (0,2)
  (corners (32,8) and (8,32) lie on it), so only the 4 tiles with x, y <= 1 remain;
* it lists a subset of the bounding-box lists, and a superset of the exact ones (the tiles
  holding a pixel where the face, rendered alone, has T < 1), on random soups, several views;
* it drops pairs on a soup of thin slanted faces."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_31419_amd import scenes as S
from tests.helpers import IDENTITY, plain_scene, tiny_scene, unit_cam


def _pairs(sc, poses, intrs, tight):
    tile, zb, face, ranges = O.bin_pairs(sc, poses, intrs, tight_tiles=tight)
    return set(zip(tile.tolist(), face.tolist())), tile, zb, face, ranges


def test_right_triangle_closed_form():
    cam = unit_cam(64, 64)
    sc = plain_scene(np.array([[[0.0, 0.0, 1.0], [63.0, 0.0, 1.0], [0.0, 63.0, 1.0]]]))
    loose, *_ = _pairs(sc, [IDENTITY], [cam], False)
    tight, *_ = _pairs(sc, [IDENTITY], [cam], True)
    assert len(loose) == 16
    want = {(y * 4 + x, 0) for y in range(4) for x in range(4) if x + y <= 3}
    assert tight == want


def test_box_is_clipped_to_the_pixel_rectangle():
    cam = unit_cam(64, 64)
    sc = plain_scene(np.array([[[8.0, 8.0, 1.0], [32.0, 8.0, 1.0], [8.0, 32.0, 1.0]]]))
    tight, *_ = _pairs(sc, [IDENTITY], [cam], True)
    assert tight == {(y * 4 + x, 0) for y in range(2) for x in range(2)}


def _exact_pairs(sc, pose, intr, base_tile=0, base_face=0):
    """(tile, face) pairs where the face, rendered alone, covers a pixel of the tile."""
    out = set()
    tx = (intr.width + 15) // 16
    for m in range(sc.n_faces):
        sub = sc.subset(np.array([m]))
        T = O.render(sub, pose, intr)[2].reshape(intr.height, intr.width)
        ys, xs = np.nonzero(T < 1.0)
        for t in set(((ys // 16) * tx + xs // 16).tolist()):
            out.add((base_tile + t, base_face + m))
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_between_exact_and_bounding_box(seed):
    sc, intr = tiny_scene(seed, n_faces=40, w=70, h=45, f=40.0, size=(0.1, 1.2))
    g = np.random.default_rng(seed)
    from tests.helpers import left_perturb
    poses = [IDENTITY, left_perturb(IDENTITY, g.normal(scale=0.05, size=6)).astype(np.float32)]
    intrs = [intr, S.Intrinsics(50, 37, 35.0, 35.0, 24.5, 18.0)]
    loose, *_ = _pairs(sc, poses, intrs, False)
    tight, tile, zb, face, ranges = _pairs(sc, poses, intrs, True)
    exact = set()
    base = 0
    for v in range(2):
        exact |= _exact_pairs(sc, poses[v], intrs[v], base, v * sc.n_faces)
        base += ((intrs[v].width + 15) // 16) * ((intrs[v].height + 15) // 16)
    assert exact <= tight <= loose
    assert len(tight) < len(loose)
    # sorted within each tile by (z bits, face) and ranges consistent, as for the loose lists
    for t in range(ranges.shape[0]):
        s, e = ranges[t]
        assert np.all(tile[s:e] == t)
        key = zb[s:e].astype(np.int64) * (1 << 32) + face[s:e]
        assert np.all(np.diff(key) > 0)


def test_thin_slanted_faces_drop_pairs():
    g = np.random.default_rng(5)
    n = 60
    c = g.uniform(10, 110, size=(n, 2))
    d = g.normal(size=(n, 2))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    perp = np.stack([-d[:, 1], d[:, 0]], axis=1)
    a = c - 40 * d
    b = c + 40 * d
    e = c + 1.5 * perp
    v = np.stack([a, b, e], axis=1)
    sc = plain_scene(np.concatenate([v, np.ones((n, 3, 1))], axis=2))
    cam = unit_cam(128, 128)
    loose, *_ = _pairs(sc, [IDENTITY], [cam], False)
    tight, *_ = _pairs(sc, [IDENTITY], [cam], True)
    exact = _exact_pairs(sc, IDENTITY, cam)
    assert exact <= tight <= loose
    assert len(tight) < 0.75 * len(loose), (len(tight), len(loose))
