"""Pins of the FP64 per-face screen statistics (projected area, dominant-pixel coverage,
visibility; the map-management tests of Sec. 3.4): the area's closed form for a frontal
triangle, and coverage / visibility against a brute force built from single-face renders
(each face rendered alone gives its alpha at every pixel as 1 - T), composited in depth order
here with the early stop."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_31419_amd import scenes as S
from tests.helpers import IDENTITY, tiny_scene


def _one_face(sc, m):
    idx = [3 * m, 3 * m + 1, 3 * m + 2]
    return S.Scene(sc.pos[:, idx].copy(), sc.col[:, idx].copy(), sc.opa[idx].copy())


def _brute(sc, pose, intr, t_min):
    """Per-face coverage and visibility by compositing single-face alphas in pure numpy."""
    M = sc.n_faces
    P = intr.width * intr.height
    alpha = np.zeros((M, P))
    for m in range(M):
        _, _, tr = O.render(_one_face(sc, m), pose, intr)
        alpha[m] = 1.0 - tr
    q, ff, rect, tiles = O.project(sc, pose, intr)
    zkey = ff[3]
    order = sorted(range(M), key=lambda m: (np.inf if np.isnan(zkey[m]) else zkey[m], m))
    T = np.ones(P)
    best_w = np.zeros(P)
    best = np.full(P, -1)
    vis = np.zeros(M, bool)
    for m in order:
        live = (T >= t_min) & (T > 0)
        a = np.where(live, alpha[m], 0.0)
        w = a * T
        upd = w > best_w
        best_w = np.where(upd, w, best_w)
        best = np.where(upd, m, best)
        vis[m] = bool(np.any(a > 0))
        T = T * (1 - a)
    cov = np.bincount(best[best >= 0], minlength=M)
    return cov, vis


def test_area_of_a_frontal_triangle():
    z, f = 2.0, 50.0
    a, b = float(np.float32(0.3)), float(np.float32(0.2))       # the legs as stored
    pos = np.array([[0.0, 0.0, z], [a, 0.0, z], [0.0, b, z]], np.float32).T
    sc = S.Scene(pos, np.full((3, 3), 0.5, np.float32), np.full(3, 0.8, np.float32))
    intr = S.Intrinsics(64, 64, f, f, 20.0, 20.0)
    area = O.face_stats(sc, IDENTITY, intr)[0]
    assert abs(area[0] - f * f * a * b / (2 * z * z)) < 1e-9 * area[0]


def test_area_is_zero_for_culled_and_offscreen_faces():
    pos = np.array([[0, 0, 0.05], [0.1, 0, 0.05], [0, 0.1, 0.05],        # in front of the near plane
                    [50, 50, 2], [51, 50, 2], [50, 51, 2]], np.float32).T  # off-screen
    sc = S.Scene(pos, np.full((3, 6), 0.5, np.float32), np.full(6, 0.8, np.float32))
    area, lo, hi, vc, vp = O.face_stats(sc, IDENTITY, S.Intrinsics(32, 32, 30.0, 30.0, 15.5, 15.5))
    assert np.all(area == 0) and np.all(hi == 0) and not vp.any()


@pytest.mark.parametrize("seed,t_min", [(1, 1e-6), (2, 1e-6), (3, 0.3), (4, 0.9)])
def test_coverage_and_visibility_match_the_brute_force(seed, t_min):
    sc, intr = tiny_scene(seed, n_faces=12, w=24, h=20, f=24.0)
    area, lo, hi, vc, vp = O.face_stats(sc, IDENTITY, intr, t_min=t_min)
    cov, vis = _brute(sc, IDENTITY, intr, t_min)
    assert np.all(lo <= cov) and np.all(cov <= hi), (lo, cov, hi)
    assert np.all(vis[vc]) and not np.any(vis & ~vp)
    assert (hi - lo).sum() <= 0.02 * max(cov.sum(), 1)          # ambiguity is rare


def test_total_coverage_is_the_number_of_touched_pixels():
    sc, intr = tiny_scene(5, n_faces=20, w=32, h=24)
    area, lo, hi, vc, vp = O.face_stats(sc, IDENTITY, intr, t_min=0.0)
    _, _, tr = O.render(sc, IDENTITY, intr)
    touched = int(np.sum(tr < 1.0))
    assert lo.sum() <= touched <= hi.sum()


def test_front_face_takes_the_coverage_of_an_identical_face_behind():
    pos = np.array([[-0.4, -0.3, 1.0], [0.5, -0.3, 1.0], [0.0, 0.5, 1.0]], np.float32).T
    back = pos * np.float32(2.0)                     # the same projection, twice as far
    sc = S.Scene(np.concatenate([back, pos], axis=1), np.full((3, 6), 0.5, np.float32),
                 np.ones(6, np.float32))
    area, lo, hi, vc, vp = O.face_stats(sc, IDENTITY, S.Intrinsics(32, 32, 30.0, 30.0, 15.5, 15.5))
    assert abs(area[0] - area[1]) <= 1e-9 * area[1]
    assert lo[0] == 0 and lo[1] > 50 and vc[0] and vc[1]


def test_early_stop_hides_a_face_behind():
    front = np.array([[-0.6, -0.5, 1.0], [0.7, -0.5, 1.0], [0.0, 0.8, 1.0]], np.float32).T
    back = np.array([[-0.05, -0.05, 2.0], [0.05, -0.05, 2.0], [0.0, 0.05, 2.0]], np.float32).T
    sc = S.Scene(np.concatenate([front, back], axis=1), np.full((3, 6), 0.5, np.float32),
                 np.ones(6, np.float32))
    intr = S.Intrinsics(32, 32, 30.0, 30.0, 15.5, 15.5)
    # the front face's alpha near its incentre is close to 1: with t_min = 0.9 every pixel of
    # the small back face has stopped before reaching it
    area, lo, hi, vc, vp = O.face_stats(sc, IDENTITY, intr, t_min=0.9)
    assert area[1] > 0 and not vp[1] and hi[1] == 0
    area, lo, hi, vc, vp = O.face_stats(sc, IDENTITY, intr, t_min=0.0)
    assert vc[1]
