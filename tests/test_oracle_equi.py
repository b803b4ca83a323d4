"""Pins of the FP64 equilateral-regulariser reference (Sec. 3.4, eq. 14): law of cosines,
angle sum, closed forms, invariances of the loss and the gradient, finite differences."""
import numpy as np
import pytest

from oracle import equi as Q


def _soup(seed, M):
    return np.random.default_rng(seed).normal(size=(3, 3 * M))


def _rot(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    return q * np.sign(np.linalg.det(q))


def test_cosines_match_the_law_of_cosines():
    pos = _soup(1, 50)
    c = Q.corner_cosines(pos)
    P = [pos[:, k::3] for k in range(3)]
    for k in range(3):
        a = np.linalg.norm(P[(k + 1) % 3] - P[(k + 2) % 3], axis=0)   # side opposite corner k
        b = np.linalg.norm(P[(k + 1) % 3] - P[k], axis=0)
        cc = np.linalg.norm(P[(k + 2) % 3] - P[k], axis=0)
        np.testing.assert_allclose(c[:, k], (b * b + cc * cc - a * a) / (2 * b * cc), atol=1e-12)


def test_angles_sum_to_pi():
    c = Q.corner_cosines(_soup(2, 40))
    np.testing.assert_allclose(np.arccos(c).sum(axis=1), np.pi, atol=1e-10)


def test_equilateral_faces_have_zero_loss_and_gradient():
    t = np.array([[0, 0, 0], [1, 0, 0], [0.5, np.sqrt(3) / 2, 0]], float).T
    pos = np.concatenate([3.7 * _rot(s) @ t + np.random.default_rng(s).normal(size=(3, 1)) for s in range(5)], axis=1)
    assert Q.e_equi(pos) < 1e-28
    assert np.abs(Q.e_equi_grad(pos)).max() < 1e-14


def test_right_isosceles_closed_form():
    pos = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float).T
    r = np.sqrt(0.5)
    assert abs(Q.e_equi(pos) - ((0 - 0.5) ** 2 + 2 * (r - 0.5) ** 2) / 3) < 1e-15


def test_invariances_of_loss_and_gradient():
    pos = _soup(3, 30)
    L = Q.e_equi(pos)
    R = _rot(4)
    assert abs(Q.e_equi(2.5 * R @ pos + np.array([[1.0], [-2.0], [0.5]])) - L) < 1e-14
    g = Q.e_equi_grad(pos)
    for m in range(30):
        x, gm = pos[:, 3 * m:3 * m + 3], g[:, 3 * m:3 * m + 3]
        np.testing.assert_allclose(gm.sum(axis=1), 0, atol=1e-13)                        # translation
        np.testing.assert_allclose(np.cross(x.T, gm.T).sum(axis=0), 0, atol=1e-13)      # rotation
        assert abs(np.sum(x * gm)) < 1e-13                                               # scale


def test_degenerate_face_contributes_nothing_but_counts():
    pos = _soup(5, 4)
    L = Q.e_equi(pos)
    deg = np.concatenate([pos, pos[:, :1].repeat(2, axis=1), pos[:, 1:2]], axis=1)      # two equal corners
    assert abs(Q.e_equi(deg) - L * 4 / 5) < 1e-15
    assert np.abs(Q.e_equi_grad(deg)[:, 12:]).max() == 0


def test_indexed_mesh_equals_the_soup_with_summed_gradients():
    g = np.random.default_rng(6)
    verts = g.normal(size=(3, 20))
    faces = np.array([g.choice(20, 3, replace=False) for _ in range(35)])
    soup = verts[:, faces.reshape(-1)]
    assert abs(Q.e_equi(verts, faces) - Q.e_equi(soup)) < 1e-15
    gs = Q.e_equi_grad(soup)
    want = np.zeros_like(verts)
    for k, vi in enumerate(faces.reshape(-1)):
        want[:, vi] += gs[:, k]
    np.testing.assert_allclose(Q.e_equi_grad(verts, faces), want, atol=1e-15)


@pytest.mark.parametrize("indexed", [False, True])
def test_gradient_matches_central_differences(indexed):
    g = np.random.default_rng(7 + indexed)
    if indexed:
        pos = g.normal(size=(3, 12))
        faces = np.array([g.choice(12, 3, replace=False) for _ in range(15)])
    else:
        pos, faces = _soup(8, 10), None
    grad = Q.e_equi_grad(pos, faces)
    h = 1e-6
    for ax in range(3):
        for i in range(pos.shape[1]):
            p1, p2 = pos.copy(), pos.copy()
            p1[ax, i] += h
            p2[ax, i] -= h
            fd = (Q.e_equi(p1, faces) - Q.e_equi(p2, faces)) / (2 * h)
            assert abs(fd - grad[ax, i]) <= 1e-7 * max(1.0, abs(fd)), (ax, i, fd, grad[ax, i])
