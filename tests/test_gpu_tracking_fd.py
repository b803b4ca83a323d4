"""Tracking stress workload (1200x680, 1M-face room soup, 90 % 0.5-2 cm / 10 % 5-20 cm faces),
checked on a seeded 5,000-face subset: the GPU's pose and vertex gradients of the L1 tracking
loss against the oracle's analytic gradient over the whole frame, and both against FP64
central differences of the oracle's forward: all six pose components, over the pixels whose
discrete rendering state (covering set, depth order, minimising edge, clamps) is the same at
both ends of every difference, with the analytic gradients (oracle and GPU backward) taken
from the same pixels; 48 sampled vertex coordinates, each difference rendered only over the
perturbed face's pixel rectangle, outside which the image cannot change.  Targets: the subset
rendered by the oracle from the pose perturbed by 1 cm / 0.5 deg."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2605_31419_amd import scenes as S
from tests import gpu_util as G
from tests.helpers import grad_close, left_perturb

pytestmark = pytest.mark.gpu
H = 1e-6


def _subset():
    w = S.workload("track_1200x680_1M")
    intr, pose, tpose = w.intr[0], w.poses[0], w.target_poses[0]
    q, f, rect, tiles = O.project(w.scene, pose, intr)
    vis = np.nonzero(tiles > 0)[0]
    g = np.random.default_rng(55)
    faces = np.sort(g.choice(vis, size=min(5000, vis.size), replace=False))
    return w.scene.subset(faces), pose, tpose, intr


def _loss(sc, pose, intr, tc, td, pix=None):
    C, D, T = O.render(sc, pose, intr, pixels=pix)
    sub_c = tc if pix is None else tc[:, pix]
    sub_d = td if pix is None else td[pix]
    L, _, _ = O.l1_seeds(C, D, sub_c, sub_d, intr.width * intr.height)
    return L


def test_tracking_subset_gradients_against_oracle_and_finite_differences():
    sc, pose, tpose, intr = _subset()
    P = intr.width * intr.height
    tcol, tdep, _ = O.render(sc, tpose, intr)
    tc, td = tcol.astype(np.float32), tdep.astype(np.float32)
    # keep every residual at least 1e-3 away from the L1 kink (same sign in FP32 and FP64)
    C0, D0, _ = O.render(sc, pose, intr)
    near = np.abs(tc - C0) < 1e-3
    tc[near] = (C0[near] + 2e-3).astype(np.float32)
    nd = np.abs(td - D0) < 1e-3
    td[nd] = (D0[nd] + 2e-3).astype(np.float32)
    L0, gcv, gdv = O.l1_seeds(C0, D0, tc, td, P)
    ref = O.backward(sc, pose, intr, gcv, gdv, None, with_abs=True)
    rp, rc, ro, rpose, conds = ref

    rast, p = G.make(sc, [intr], [pose])
    rast.bin_and_sort(p)
    loss = torch.zeros(1, device="cuda")
    out = rast.train_l1(p, G.to_dev(tc), G.to_dev(td), loss=loss)
    torch.cuda.synchronize()
    gp, gc, go, gpose = [x.cpu().numpy().astype(np.float64) for x in out]
    gp = gp.reshape(3, -1)
    assert abs(loss.item() - L0) <= 1e-5 * abs(L0)
    for nm, a, b, cond in [("pos", gp, rp, conds[0]), ("col", gc, rc, conds[1]), ("opa", go, ro, conds[2]),
                           ("pose", gpose, rpose, None)]:
        ok, msg, _ = grad_close(a, b, name=nm, cond=cond)
        print("  " + msg, flush=True)
        assert ok, msg

    # FP64 central differences of the oracle forward for the pose, over the stable pixels:
    # same rendering state and same L1 residual signs at both ends of every difference (steep
    # faces move a pixel's colour by several 1e-3 per 1e-6 step, enough to cross the L1 kink)
    st0 = O.state(sc, pose, intr)
    s0c, s0d = np.sign(C0 - tc), np.sign(D0 - td)
    stable = np.ones(P, bool)
    for k in range(6):
        for sgn in (1.0, -1.0):
            tau = np.zeros(6); tau[k] = sgn * H
            pk = left_perturb(pose, tau)
            Ck, Dk, _ = O.render(sc, pk, intr)
            stable &= O.state(sc, pk, intr) == st0
            stable &= (np.sign(Ck - tc) == s0c).all(0) & (np.sign(Dk - td) == s0d)
    keep = np.nonzero(stable)[0]
    print(f"  pose differences over {keep.size} of {P} pixels", flush=True)
    assert keep.size >= 0.99 * P
    gcm, gdm = gcv * stable, gdv * stable
    rpose_m = O.backward(sc, pose, intr, gcm, gdm, None)[3]
    rast.forward(p)
    gpose_m = rast.backward(p, G.to_dev(gcm.astype(np.float32)), G.to_dev(gdm.astype(np.float32)))[3]
    gpose_m = gpose_m.cpu().numpy().astype(np.float64)
    scale = np.abs(rpose_m).max()
    for k in range(6):
        tau = np.zeros(6); tau[k] = H
        fd = (_loss(sc, left_perturb(pose, tau), intr, tc, td, keep) -
              _loss(sc, left_perturb(pose, -tau), intr, tc, td, keep)) / (2 * H)
        print(f"  pose[{k}] gpu {gpose_m[k]:.6e} oracle {rpose_m[k]:.6e} fd {fd:.6e}", flush=True)
        assert abs(fd - rpose_m[k]) <= 1e-5 * abs(rpose_m[k]) + 1e-8 * scale
        assert abs(fd - gpose_m[k]) <= 1e-3 * abs(fd) + 1e-5 * scale

    # vertex coordinates: finite differences over the perturbed face's pixel rectangle
    g = np.random.default_rng(56)
    q, f, rect, tiles = O.project(sc, pose, intr)
    cand = np.nonzero(tiles > 0)[0]
    picks = g.choice(cand, size=16, replace=False)
    pos64 = sc.pos.astype(np.float64)
    checked = 0
    for m in picks:
        u0, u1, v0, v1 = rect[:, m]
        pad = 2
        ys, xs = np.mgrid[max(v0 - pad, 0):min(v1 + pad, intr.height - 1) + 1,
                          max(u0 - pad, 0):min(u1 + pad, intr.width - 1) + 1]
        pix = (ys * intr.width + xs).reshape(-1).astype(np.int64)
        for a in range(3):
            vi = 3 * m + g.integers(0, 3)
            pp = pos64.copy(); pp[a, vi] += H
            pm = pos64.copy(); pm[a, vi] -= H
            sp = S.Scene(pp, sc.col, sc.opa); sm = S.Scene(pm, sc.col, sc.opa)
            st0 = O.state(sc, pose, intr, pixels=pix)
            if not (np.array_equal(O.state(sp, pose, intr, pixels=pix), st0)
                    and np.array_equal(O.state(sm, pose, intr, pixels=pix), st0)):
                continue
            fd = (_loss(sp, pose, intr, tc, td, pix) - _loss(sm, pose, intr, tc, td, pix)) / (2 * H)
            scale = np.abs(rp).max()
            assert abs(fd - rp[a, vi]) <= 1e-4 * abs(rp[a, vi]) + 1e-7 * scale, (m, a, fd, rp[a, vi])
            assert abs(fd - gp[a, vi]) <= 1e-3 * abs(fd) + 1e-5 * scale + 2e-6 * np.reshape(conds[0], (3, -1))[a, vi], (m, a, fd, gp[a, vi])
            checked += 1
    assert checked >= 24, checked
