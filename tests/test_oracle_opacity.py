"""Pins of the minimum face-opacity rule (the Mesh Splatting variant the paper departs from in
Sec. 3.1 and compares with in its ablation): the rendered alpha of a single face against the
closed form, the opacity gradient against FP64 central differences (all of it on the
lowest-opacity vertex), and the tie convention."""
import numpy as np

from oracle import oracle as O
from paper_2605_31419_amd import scenes as S
from tests.helpers import IDENTITY, tiny_scene

H = 1e-6


def _one_face(opa):
    pos = np.array([[-0.4, -0.3, 1.5], [0.5, -0.25, 1.6], [0.0, 0.45, 1.4]]).T
    intr = S.Intrinsics(24, 20, 24.0, 24.0, 11.5, 9.5)
    return S.Scene(pos, np.full((3, 3), 0.5), np.asarray(opa, np.float64)), intr


def test_single_face_alpha_is_the_minimum_times_the_window():
    sc, intr = _one_face([0.9, 0.3, 0.6])
    _, _, t_min = O.render(sc, IDENTITY, intr, opacity_min=True)
    _, _, t_mean = O.render(sc, IDENTITY, intr)
    cov = t_mean < 1.0
    assert cov.sum() > 20
    np.testing.assert_allclose((1.0 - t_min[cov]) / (1.0 - t_mean[cov]), 0.3 / 0.6, rtol=1e-12)
    assert np.all(t_min[~cov] == 1.0)


def test_opacity_gradient_goes_to_the_lowest_vertex_and_matches_differences():
    sc32, intr = tiny_scene(8, n_faces=6, w=28, h=22, f=26.0)
    g = np.random.default_rng(8)
    sc = S.Scene(sc32.pos.astype(np.float64), sc32.col.astype(np.float64), g.uniform(0.3, 0.9, size=sc32.n_vertices))
    P = intr.width * intr.height
    wC, wD, wT = g.normal(size=(3, P)), g.normal(size=P), g.normal(size=P)
    gopa = O.backward(sc, IDENTITY, intr, wC, wD, wT, opacity_min=True)[2]

    def loss(s):
        C, D, T = O.render(s, IDENTITY, intr, opacity_min=True)
        return float((wC * C).sum() + (wD * D).sum() + (wT * T).sum())

    for m in range(sc.n_faces):
        o = sc.opa[3 * m:3 * m + 3]
        kmin = int(np.argmin(o))
        for k in range(3):
            i = 3 * m + k
            op, om = sc.opa.copy(), sc.opa.copy()
            op[i] += H
            om[i] -= H
            fd = (loss(S.Scene(sc.pos, sc.col, op)) - loss(S.Scene(sc.pos, sc.col, om))) / (2 * H)
            if k != kmin:
                assert gopa[i] == 0.0 and abs(fd) < 1e-9, (m, k, gopa[i], fd)
            else:
                assert abs(fd - gopa[i]) <= 1e-6 * max(1.0, abs(fd)), (m, k, gopa[i], fd)


def test_ties_send_the_gradient_to_the_lowest_index():
    sc, intr = _one_face([0.5, 0.5, 0.8])
    P = intr.width * intr.height
    gopa = O.backward(sc, IDENTITY, intr, np.ones((3, P)), np.zeros(P), np.zeros(P), opacity_min=True)[2]
    assert gopa[0] != 0.0 and gopa[1] == 0.0 and gopa[2] == 0.0
