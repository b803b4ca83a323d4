"""Pins of the oracle's analytic gradient (Sec. 3.3, eqs. 5-7) to FP64 central differences of
its own forward on tiny scenes, plus exact identities tying the pose gradient to the vertex
gradients and the opacity-mean rule (Sec. 3.1).

Rejection rule: a parameter whose finite difference crosses a discontinuity of the rendering
(covering set, depth order, maximising edge, window clamp, steep edge band when sigma < 1)
is excluded; the test reports how many were excluded and requires most to remain.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_31419_amd import scenes as S
from tests.helpers import IDENTITY, left_perturb, tiny_scene

H = 1e-6


def _loss(sc, pose, intr, sigma, wC, wD, wT):
    C, D, T = O.render(sc, pose, intr, sigma=sigma)
    return float((wC * C).sum() + (wD * D).sum() + (wT * T).sum())


def _scene64(sc):
    return S.Scene(sc.pos.astype(np.float64), sc.col.astype(np.float64), sc.opa.astype(np.float64), sc.faces)


def _random_pose(g):
    tau = np.concatenate([g.normal(scale=0.05, size=3), g.normal(scale=0.05, size=3)])
    return left_perturb(IDENTITY, tau)


@pytest.mark.parametrize("sigma,seed", [(1.0, 1), (0.5, 2), (2.0, 3), (1.0, 4)])
def test_gradients_match_finite_differences(sigma, seed):
    sc32, intr = tiny_scene(seed, n_faces=10, w=32, h=24)
    sc = _scene64(sc32)
    g = np.random.default_rng(seed)
    pose = _random_pose(g)
    P = intr.width * intr.height
    wC, wD, wT = g.normal(size=(3, P)), g.normal(size=P), g.normal(size=P)
    gpos, gcol, gopa, gpose = O.backward(sc, pose, intr, wC, wD, wT, sigma=sigma)
    base_state = O.state(sc, pose, intr, sigma=sigma)

    def fd(make):
        sp, pp = make(+H)
        sm, pm = make(-H)
        if not (np.array_equal(O.state(sp, pp, intr, sigma=sigma), base_state)
                and np.array_equal(O.state(sm, pm, intr, sigma=sigma), base_state)):
            return None
        return (_loss(sp, pp, intr, sigma, wC, wD, wT) - _loss(sm, pm, intr, sigma, wC, wD, wT)) / (2 * H)

    checked = rejected = 0
    worst = 0.0
    scale = max(np.abs(gpos).max(), np.abs(gcol).max(), np.abs(gopa).max(), np.abs(gpose).max())

    def check(an, num):
        nonlocal checked, rejected, worst
        if num is None:
            rejected += 1
            return
        checked += 1
        err = abs(num - an) / (abs(an) + 1e-6 * scale)
        worst = max(worst, err)
        assert err < 1e-5, (an, num)

    N = sc.n_vertices
    for i in range(N):
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
    assert np.abs(gpos).max() > 0 and np.abs(gpose).max() > 0
    print(f"sigma={sigma}: {checked} parameters checked, {rejected} rejected, worst rel err {worst:.2e}")


def _stacked_scene(seed, n=6, w=24, h=20, f=20.0):
    """Large faces stacked in depth over the whole image (every pixel sees several layers)."""
    g = np.random.default_rng(seed)
    intr = S.Intrinsics(w, h, f, f, (w - 1) / 2.0, (h - 1) / 2.0)
    verts = []
    for i in range(n):
        z = 1.0 + 0.4 * i + g.uniform(0, 0.1)
        c = g.uniform(-0.1, 0.1, size=2)
        ang = g.uniform(0, 2 * np.pi) + np.array([0, 2.1, 4.2])
        rad = z * g.uniform(0.9, 1.3)
        verts.append(np.stack([c[0] + rad * np.cos(ang), c[1] + rad * np.sin(ang), z + g.uniform(-0.05, 0.05, 3)], 1))
    sc = S.Scene(np.ascontiguousarray(np.concatenate(verts).T), g.uniform(0, 1, (3, 3 * n)),
                 g.uniform(0.3, 0.8, 3 * n), None)
    return sc, intr


@pytest.mark.parametrize("sigma", [1.0, 2.0])
def test_gradients_with_deep_overlap(sigma):
    """Finite differences where every pixel composites several layers, so the behind-colour
    accumulation of the backward (eq. 4 derivative) is exercised beyond one layer."""
    sc, intr = _stacked_scene(5)
    g = np.random.default_rng(5)
    pose = _random_pose(g)
    P = intr.width * intr.height
    wC, wD, wT = g.normal(size=(3, P)), g.normal(size=P), g.normal(size=P)
    gpos, gcol, gopa, gpose = O.backward(sc, pose, intr, wC, wD, wT, sigma=sigma)
    C, D, T = O.render(sc, pose, intr, sigma=sigma)
    assert (T < 0.7).mean() > 0.5                        # deep overlap indeed
    base = O.state(sc, pose, intr, sigma=sigma)
    checked = 0
    for k in range(sc.n_vertices):
        for (arr, an) in ((sc.col, gcol), (sc.pos, gpos)):
            for a in range(3):
                def mk(h, arr=arr, a=a, k=k):
                    x = arr.copy(); x[a, k] += h
                    return S.Scene(x, sc.col, sc.opa) if arr is sc.pos else S.Scene(sc.pos, x, sc.opa)
                sp, sm = mk(H), mk(-H)
                if not (np.array_equal(O.state(sp, pose, intr, sigma=sigma), base)
                        and np.array_equal(O.state(sm, pose, intr, sigma=sigma), base)):
                    continue
                num = (_loss(sp, pose, intr, sigma, wC, wD, wT) - _loss(sm, pose, intr, sigma, wC, wD, wT)) / (2 * H)
                assert abs(num - an[a, k]) <= 1e-5 * abs(an[a, k]) + 1e-7 * np.abs(an).max(), (k, a, num, an[a, k])
                checked += 1
    for k in range(sc.n_vertices):
        def mko(h, k=k):
            o = sc.opa.copy(); o[k] += h
            return S.Scene(sc.pos, sc.col, o)
        num = (_loss(mko(H), pose, intr, sigma, wC, wD, wT) - _loss(mko(-H), pose, intr, sigma, wC, wD, wT)) / (2 * H)
        assert abs(num - gopa[k]) <= 1e-5 * abs(gopa[k]) + 1e-7 * np.abs(gopa).max()
    assert checked > 50


@pytest.mark.parametrize("seed", [7, 8])
def test_pose_gradient_identities(seed):
    """Eq. (7): dL/drho = sum_i dL/dv_C,i = R sum_i dL/dv_W,i and dL/dtheta = sum_i v_C,i x
    dL/dv_C,i with dL/dv_C = R dL/dv_W -- exact ties between the pose reduction and the
    vertex gradients."""
    sc32, intr = tiny_scene(seed, n_faces=15, w=40, h=30)
    sc = _scene64(sc32)
    g = np.random.default_rng(seed)
    pose = _random_pose(g)
    P = intr.width * intr.height
    gpos, gcol, gopa, gpose = O.backward(sc, pose, intr, g.normal(size=(3, P)), g.normal(size=P),
                                         g.normal(size=P))
    R = pose[:9].reshape(3, 3)
    t = pose[9:]
    gC = R @ gpos                                   # dL/dv_C per vertex [3, N]
    vC = R @ sc.pos + t[:, None]
    np.testing.assert_allclose(gpose[:3], gC.sum(axis=1), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(gpose[3:], np.cross(vC.T, gC.T).sum(axis=0), rtol=1e-10, atol=1e-12)


def test_opacity_mean_rule():
    """Sec. 3.1: o_F is the mean of the three vertex opacities, so in a soup all three
    vertices of a face receive identical opacity gradients."""
    sc, intr = tiny_scene(9, n_faces=20)
    g = np.random.default_rng(9)
    P = intr.width * intr.height
    _, _, gopa, _ = O.backward(sc, IDENTITY, intr, g.normal(size=(3, P)), g.normal(size=P), None)
    go = gopa.reshape(-1, 3)
    np.testing.assert_allclose(go[:, 0], go[:, 1], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(go[:, 0], go[:, 2], rtol=1e-12, atol=1e-15)
    assert np.abs(go).max() > 0


def test_pixel_subsets_add_up():
    """Backward contributions are additive over pixels: the gradient from a pixel partition
    sums to the full-frame gradient (what sampled-pixel checks rely on)."""
    sc, intr = tiny_scene(10, n_faces=12)
    g = np.random.default_rng(10)
    P = intr.width * intr.height
    wC, wD, wT = g.normal(size=(3, P)), g.normal(size=P), g.normal(size=P)
    full = O.backward(sc, IDENTITY, intr, wC, wD, wT)
    idx = g.permutation(P)
    a, b = np.sort(idx[: P // 3]), np.sort(idx[P // 3:])
    pa = O.backward(sc, IDENTITY, intr, wC[:, a], wD[a], wT[a], pixels=a)
    pb = O.backward(sc, IDENTITY, intr, wC[:, b], wD[b], wT[b], pixels=b)
    for x, y, z in zip(full, pa, pb):
        np.testing.assert_allclose(x, y + z, rtol=1e-10, atol=1e-13)


def test_conditioning_sums_bound_the_gradient():
    """The per-element sums of absolute per-pixel contributions bound |gradient| (triangle
    inequality) and equal it when a single pixel contributes."""
    sc, intr = tiny_scene(12, n_faces=15)
    g = np.random.default_rng(12)
    P = intr.width * intr.height
    wC, wD, wT = g.normal(size=(3, P)), g.normal(size=P), g.normal(size=P)
    gp, gc, go, _, (ap, ac, ao) = O.backward(sc, IDENTITY, intr, wC, wD, wT, with_abs=True)
    for x, a in ((gp, ap), (gc, ac), (go, ao)):
        assert np.all(a >= 0) and np.all(np.abs(x) <= a * (1 + 1e-12) + 1e-15)
    C, D, T = O.render(sc, IDENTITY, intr)
    pix = np.array([int(np.argmin(T))])
    gp1, gc1, go1, _, (ap1, ac1, ao1) = O.backward(sc, IDENTITY, intr, wC[:, pix], wD[pix], wT[pix], pixels=pix,
                                                   with_abs=True)
    np.testing.assert_allclose(np.abs(gc1), ac1, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(np.abs(go1), ao1, rtol=1e-12, atol=1e-15)
