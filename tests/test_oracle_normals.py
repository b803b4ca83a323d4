"""Pins of the FP64 normal-supervision reference (Sec. 3.4: sensor normals from depth, E_norm):
sensor normals of analytic planes, the rendered normal map of a single face, the loss's
special cases, and FP64 central differences of the gradient (positions, opacities, pose)."""
import numpy as np
import pytest

from oracle import normals as NR
from oracle import oracle as O
from paper_2605_31419_amd import scenes as S
from tests.helpers import IDENTITY, left_perturb, tiny_scene

H = 1e-6


def _plane_depth(n, d, intr):
    """Depth of the plane n . x = d seen through the pinhole intr."""
    v, u = np.mgrid[0:intr.height, 0:intr.width].astype(np.float64)
    ray = np.stack([(u - intr.cx) / intr.fx, (v - intr.cy) / intr.fy, np.ones_like(u)])
    return d / np.tensordot(n, ray, axes=1)


@pytest.mark.parametrize("n", [(0.0, 0.0, 1.0), (0.3, -0.2, 0.93), (-0.5, 0.4, 0.77)])
def test_sensor_normals_of_a_plane_are_its_normal(n):
    n = np.asarray(n) / np.linalg.norm(n)
    intr = S.Intrinsics(20, 15, 18.0, 17.0, 9.3, 7.1)
    nb, valid = NR.sensor_normals(_plane_depth(n, 2.0, intr), intr)
    assert valid[1:-1, 1:-1].all() and not valid[0].any() and not valid[:, -1].any()
    np.testing.assert_allclose(nb[:, valid].T, np.tile(n, (valid.sum(), 1)), atol=1e-12)


def test_sensor_normals_skip_pixels_next_to_missing_depth():
    intr = S.Intrinsics(12, 10, 10.0, 10.0, 5.5, 4.5)
    d = np.full((10, 12), 2.0)
    d[4, 6] = 0.0
    nb, valid = NR.sensor_normals(d, intr)
    assert not valid[4, 6] and not valid[4, 5] and not valid[4, 7] and not valid[3, 6] and not valid[5, 6]
    assert valid[4, 4] and valid[2, 6]


def test_rendered_normal_of_one_face_is_alpha_times_its_normal():
    sc, intr = tiny_scene(1, n_faces=1, w=24, h=20, f=24.0)
    pose = left_perturb(IDENTITY, np.array([0.02, -0.01, 0.03, 0.1, -0.05, 0.08]))
    N = NR.render_normals(sc, pose, intr)
    _, _, T = O.render(sc, pose, intr)
    nw = NR.face_normals(sc.pos)[:, 0]
    R = np.asarray(pose, np.float64)[:9].reshape(3, 3)
    np.testing.assert_allclose(N, np.outer(R @ nw, 1.0 - T), atol=1e-12)
    assert abs(np.linalg.norm(nw) - 1) < 1e-12


def test_loss_special_cases():
    sc, intr = tiny_scene(2, n_faces=6, w=24, h=20, f=24.0)
    P = intr.width * intr.height
    valid = np.zeros(P, bool)
    assert NR.e_norm(sc, IDENTITY, intr, np.zeros((3, P)), valid) == 0.0
    # supervision equal to the rendered map itself: the loss is the mean of 1 - |N|^2
    N = NR.render_normals(sc, IDENTITY, intr)
    valid[:] = True
    assert abs(NR.e_norm(sc, IDENTITY, intr, N, valid) - np.mean(1 - np.sum(N * N, axis=0))) < 1e-12


@pytest.mark.parametrize("seed", [3, 4])
def test_gradient_matches_central_differences(seed):
    sc32, intr = tiny_scene(seed, n_faces=8, w=28, h=22, f=26.0)
    sc = S.Scene(sc32.pos.astype(np.float64), sc32.col.astype(np.float64), sc32.opa.astype(np.float64))
    g = np.random.default_rng(seed)
    pose = left_perturb(IDENTITY, g.normal(scale=0.04, size=6))
    P = intr.width * intr.height
    nb = g.normal(size=(3, P))
    nb /= np.linalg.norm(nb, axis=0)
    valid = g.uniform(size=P) < 0.8
    gpos, gopa, gpose = NR.e_norm_grad(sc, pose, intr, nb, valid)
    base = O.state(sc, pose, intr)
    scale = max(np.abs(gpos).max(), np.abs(gopa).max(), np.abs(gpose).max())
    checked = rejected = 0

    def fd(make):
        sp, pp = make(+H)
        sm, pm = make(-H)
        if not (np.array_equal(O.state(sp, pp, intr), base) and np.array_equal(O.state(sm, pm, intr), base)):
            return None
        return (NR.e_norm(sp, pp, intr, nb, valid) - NR.e_norm(sm, pm, intr, nb, valid)) / (2 * H)

    def check(an, num):
        nonlocal checked, rejected
        if num is None:
            rejected += 1
            return
        checked += 1
        assert abs(num - an) <= 1e-5 * (abs(an) + 1e-4 * scale), (an, num)

    for i in range(sc.n_vertices):
        for a in range(3):
            def mk(h, i=i, a=a):
                p = sc.pos.copy(); p[a, i] += h
                return S.Scene(p, sc.col, sc.opa), pose
            check(gpos[a, i], fd(mk))
        def mko(h, i=i):
            o = sc.opa.copy(); o[i] += h
            return S.Scene(sc.pos, sc.col, o), pose
        check(gopa[i], fd(mko))
    for k in range(6):
        def mkp(h, k=k):
            t = np.zeros(6); t[k] = h
            return sc, left_perturb(pose, t)
        check(gpose[k], fd(mkp))
    assert checked >= 0.8 * (checked + rejected), (checked, rejected)


def test_per_face_exponents_reach_the_normal_map():
    """Every face at exponent 2 with the global exponent 1 gives the normal map, loss and
    gradients of the global exponent 2 (the normal map blends with the faces' own windows);
    exponents that differ per face change the map."""
    sc, intr = tiny_scene(5, n_faces=10, w=28, h=22, f=26.0)
    g = np.random.default_rng(5)
    pose = left_perturb(IDENTITY, g.normal(scale=0.03, size=6))
    P = intr.width * intr.height
    nb = g.normal(size=(3, P))
    nb /= np.linalg.norm(nb, axis=0)
    valid = g.uniform(size=P) < 0.8
    two = S.Scene(sc.pos, sc.col, sc.opa, None, np.full(sc.n_faces, 2.0))
    np.testing.assert_allclose(NR.render_normals(two, pose, intr, sigma=1.0),
                               NR.render_normals(sc, pose, intr, sigma=2.0), atol=1e-14)
    assert abs(NR.e_norm(two, pose, intr, nb, valid, sigma=1.0) - NR.e_norm(sc, pose, intr, nb, valid, sigma=2.0)) < 1e-14
    for a, b in zip(NR.e_norm_grad(two, pose, intr, nb, valid, sigma=1.0),
                    NR.e_norm_grad(sc, pose, intr, nb, valid, sigma=2.0)):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)
    mixed = S.Scene(sc.pos, sc.col, sc.opa, None, g.uniform(0.5, 2.5, sc.n_faces))
    assert np.abs(NR.render_normals(mixed, pose, intr) - NR.render_normals(sc, pose, intr)).max() > 1e-3
