"""Pins of the oracle's perspective-correct variant (colour interpolated with the
perspective-correct barycentrics mu_i = (lambda_i / z_i) / sum_j lambda_j / z_j, depth D taken
from the face's plane along the pixel's ray, 1 / sum_j lambda_j / z_j; the affine screen-space
reading of Sec. 3.1 and eq. 4 is the default):

* the ray identity: with each vertex's colour set to its own camera-space position and opacity
  1, a single tilted face's colour at a covered pixel is the point where the pixel's ray meets
  the face's plane, zp ((u - cx)/fx, (v - cy)/fy, 1), and its depth is that zp -- pure 3D
  geometry, independent of how the weights are computed;
* faces parallel to the image plane give the affine images (z_i all equal);
* partition of unity: white vertices give C = 1 - T;
* FP64 central differences of every gradient."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_31419_amd import scenes as S
from tests.helpers import IDENTITY, left_perturb, plain_scene, tiny_scene

H = 1e-6


def _cam():
    return S.Intrinsics(64, 48, 50.0, 55.0, 31.5, 23.5)


def test_ray_meets_the_face_plane():
    cam = _cam()
    g = np.random.default_rng(3)
    for _ in range(5):
        c = np.array([g.uniform(-0.3, 0.3), g.uniform(-0.2, 0.2), g.uniform(1.5, 3.0)])
        v = c + g.normal(scale=1.0, size=(3, 3)) * np.array([1.0, 1.0, 0.8])
        v[:, 2] = np.maximum(v[:, 2], 0.6)
        sc = plain_scene(v[None], col=v[None], opa=np.ones((1, 3)))    # colour of vertex i = its position
        C, D, T = O.render(sc, IDENTITY, cam, perspective=True)
        a = 1.0 - T
        inside = a > 1e-3
        assert inside.sum() > 5
        P = np.arange(cam.width * cam.height)
        u, w = (P % cam.width).astype(float), (P // cam.width).astype(float)
        zp = D[inside] / a[inside]
        ray = np.stack([(u - cam.cx) / cam.fx, (w - cam.cy) / cam.fy, np.ones_like(u)])[:, inside]
        np.testing.assert_allclose(C[:, inside] / a[inside], zp * ray, rtol=1e-9, atol=1e-9)
        # zp lies on the face's plane (through the float32 vertices the oracle received)
        v32 = sc.pos.astype(np.float64).T
        nrm = np.cross(v32[1] - v32[0], v32[2] - v32[0])
        np.testing.assert_allclose(nrm @ (zp * ray - v32[0][:, None]), 0.0, atol=1e-9)


def test_fronto_parallel_faces_give_the_affine_images():
    g = np.random.default_rng(4)
    n = 30
    xy = g.uniform(-0.6, 0.6, size=(n, 1, 2)) + g.uniform(-0.15, 0.15, size=(n, 3, 2))
    z = g.uniform(1.0, 3.0, size=(n, 1, 1)) * np.ones((n, 3, 1))
    sc = plain_scene(np.concatenate([xy * z, z], axis=2), col=g.uniform(0, 1, (n, 3, 3)), opa=g.uniform(0.3, 1, (n, 3)))
    cam = _cam()
    for a, b in zip(O.render(sc, IDENTITY, cam), O.render(sc, IDENTITY, cam, perspective=True)):
        np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-12)


def test_white_faces_partition_of_unity():
    sc0, intr = tiny_scene(9, n_faces=20, w=40, h=30)
    sc = S.Scene(sc0.pos, np.ones_like(sc0.col), sc0.opa)
    C, D, T = O.render(sc, IDENTITY, intr, perspective=True)
    for ch in range(3):
        np.testing.assert_allclose(C[ch], 1.0 - T, atol=1e-12)


@pytest.mark.parametrize("seed", [11, 12])
def test_gradients_match_finite_differences(seed):
    sc32, intr = tiny_scene(seed, n_faces=10, w=32, h=24)
    sc = S.Scene(sc32.pos.astype(np.float64), sc32.col.astype(np.float64), sc32.opa.astype(np.float64))
    g = np.random.default_rng(seed)
    pose = left_perturb(IDENTITY, np.concatenate([g.normal(scale=0.05, size=3), g.normal(scale=0.05, size=3)]))
    P = intr.width * intr.height
    wC, wD, wT = g.normal(size=(3, P)), g.normal(size=P), g.normal(size=P)
    gpos, gcol, gopa, gpose = O.backward(sc, pose, intr, wC, wD, wT, perspective=True)
    base = O.state(sc, pose, intr)

    def loss(s, p):
        C, D, T = O.render(s, p, intr, perspective=True)
        return float((wC * C).sum() + (wD * D).sum() + (wT * T).sum())

    def fd(make):
        sp, pp = make(+H)
        sm, pm = make(-H)
        if not (np.array_equal(O.state(sp, pp, intr), base) and np.array_equal(O.state(sm, pm, intr), base)):
            return None
        return (loss(sp, pp) - loss(sm, pm)) / (2 * H)

    scale = max(np.abs(gpos).max(), np.abs(gcol).max(), np.abs(gpose).max())
    checked = rejected = 0

    def check(an, num):
        nonlocal checked, rejected
        if num is None:
            rejected += 1
            return
        checked += 1
        assert abs(num - an) <= 1e-5 * (abs(an) + 1e-6 * scale), (an, num)

    for i in range(sc.n_vertices):
        for a in range(3):
            def mk(h, i=i, a=a):
                p = sc.pos.copy(); p[a, i] += h
                return S.Scene(p, sc.col, sc.opa), pose
            check(gpos[a, i], fd(mk))
            def mkc(h, i=i, a=a):
                c = sc.col.copy(); c[a, i] += h
                return S.Scene(sc.pos, c, sc.opa), pose
            check(gcol[a, i], fd(mkc))
        def mko(h, i=i):
            o = sc.opa.copy(); o[i] += h
            return S.Scene(sc.pos, sc.col, o), pose
        check(gopa[i], fd(mko))
    for k in range(6):
        def mkp(h, k=k):
            tau = np.zeros(6); tau[k] = h
            return sc, left_perturb(pose, tau)
        check(gpose[k], fd(mkp))
    assert checked > 0.8 * (checked + rejected), (checked, rejected)
    print(f"seed {seed}: {checked} checked, {rejected} rejected")
