"""GPU parity of the one-binning mapping step (Sec. 3.4): the photometric and depth terms
(eqs. 8 and 10 with D-SSIM) and the normal term on the binning of the scene's colours, with the
face normals composited as three more channels of the forward walk and back-propagated in the
same backward walk (``tsr_render_train_mapping``).

References: the oracle's L1 + 0.2 D-SSIM seeds of the oracle render pushed through the oracle
backward, plus w_norm times the FP64 normal-loss gradient of the normal reference (rasteriser
backward with the world normals as colours, the normalised-cross-product chain and the rotation
term).  Tolerances as the photometric and normal steps: images within 1e-4, normal map within
1e-5, photometric loss within 1e-5 relative + 2e-5, normal loss within 1e-5 relative, gradients
by the backward's bar (1e-3 relative, with the photometric conditioning allowance)."""
import numpy as np
import pytest
import torch

from oracle import dssim as D
from oracle import normals as NR
from oracle import oracle as O
from paper_2605_31419_amd import raster
from paper_2605_31419_amd import scenes as S
from tests import gpu_util as G
from tests import test_gpu_parity as PAR
from tests.helpers import IDENTITY, grad_close, left_perturb, tiny_scene

pytestmark = pytest.mark.gpu

W_SSIM, W_NORM = 0.2, 0.05
IMG_TOL = 1e-4


def _say(*a):
    print(*a, flush=True)


def _normal_targets(seed, n_pix, frac_valid=0.8):
    g = np.random.default_rng(seed)
    nb = g.normal(size=(3, n_pix))
    nb /= np.linalg.norm(nb, axis=0)
    valid = g.uniform(size=n_pix) < frac_valid
    nb[:, ~valid] = 0.0
    return nb.astype(np.float32), valid


def _run(sc, poses, intrs, seed, sigma=1.0, perspective=False, face_sigma=False):
    rast = raster.Rasterizer(raster.DeviceScene.from_numpy(sc), intrs,
                             raster.Params(sigma=sigma, perspective=perspective))
    p = raster.poses_tensor(poses)
    rast.fit(p)
    n_views = len(poses)
    tcs, tds, tns, ocs, lref, nlref, gcs, gds, nmaps = [], [], [], [], [], [], [], [], []
    for v in range(n_views):
        it = intrs[v]
        Wd, H = it.width, it.height
        oc, od, _ = O.render(sc, poses[v], it, sigma=sigma, perspective=perspective)
        tc, td, _ = PAR._nudged_targets(oc, od, seed + v, None)
        L, gcv, gdv = O.l1_seeds(oc, od, tc, td, Wd * H)
        c3, t3 = np.asarray(oc, np.float64).reshape(3, H, Wd), tc.astype(np.float64).reshape(3, H, Wd)
        lref.append(L + W_SSIM * D.dssim(c3, t3))
        gcs.append(gcv + W_SSIM * D.dssim_grad(c3, t3).reshape(gcv.shape))
        gds.append(gdv)
        nb, valid = _normal_targets(seed + 50 + v, Wd * H)
        if sigma < 1.0:
            # the steep-edge band and ridges (as the backward parity tests): no normal target
            # there, so the normal seeds vanish on both sides
            m = PAR._steep_masks(sc, [poses[v]], [it], sigma)[0]
            nb[:, m] = 0.0
            valid = valid & ~m
        nlref.append(W_NORM * NR.e_norm(sc, poses[v], it, nb.astype(np.float64), valid, sigma=sigma))
        nmaps.append(NR.render_normals(sc, poses[v], it, sigma=sigma))
        tcs.append(tc); tds.append(td); tns.append((nb, valid)); ocs.append(oc)
    rast.bin_and_sort(p)
    P = rast.total_pixels
    color = torch.empty(3 * P, device="cuda")
    depth = torch.empty(P, device="cuda")
    nmap = torch.empty(3 * P, device="cuda")
    loss = torch.zeros(n_views, device="cuda")
    nloss = torch.zeros(n_views, device="cuda")
    out = rast.train_mapping(p, G.to_dev(np.concatenate([t.reshape(-1) for t in tcs])),
                             G.to_dev(np.concatenate([t.reshape(-1) for t in tds])),
                             G.to_dev(np.concatenate([t[0].reshape(-1) for t in tns])), w_ssim=W_SSIM, w_norm=W_NORM,
                             color=color, depth=depth, normal_map=nmap, loss=loss, loss_norm=nloss)
    torch.cuda.synchronize()
    got = [x.cpu().numpy().astype(np.float64) for x in out]
    if face_sigma:
        got.append(rast.grad_face_sigma.cpu().numpy().astype(np.float64))
    _say(f"  loss {loss.cpu().numpy()} ref {np.array(lref)}; normal loss {nloss.cpu().numpy()} ref {np.array(nlref)}")
    np.testing.assert_allclose(loss.cpu().numpy(), lref, rtol=1e-5, atol=2e-5)
    np.testing.assert_allclose(nloss.cpu().numpy(), nlref, rtol=1e-5, atol=1e-9)
    cs = G.per_view(rast, color.cpu().numpy(), 3)
    ns = G.per_view(rast, nmap.cpu().numpy(), 3)
    for v in range(n_views):
        assert np.abs(cs[v] - ocs[v]).max() <= IMG_TOL
        err = np.abs(ns[v] - nmaps[v]).max()
        assert err <= 1e-5, (v, err)
    # photometric part: the oracle backward of the seeds, with its conditioning sums
    acc, cond, gposes = None, None, []
    gsig = np.zeros(sc.n_faces)
    for v in range(n_views):
        res = O.backward(sc, poses[v], intrs[v], gcs[v], gds[v], None, sigma=sigma, with_abs=True,
                         perspective=perspective, want_sigma=face_sigma)
        if face_sigma:
            gp, gc, go, gpose, gs, ab = res
            gsig += gs
        else:
            gp, gc, go, gpose, ab = res
        acc = [gp, gc, go] if acc is None else [a + b for a, b in zip(acc, [gp, gc, go])]
        cond = list(ab[:3]) if cond is None else [c + x for c, x in zip(cond, ab[:3])]
        gposes.append(np.asarray(gpose, np.float64).reshape(6))
    # normal part
    for v in range(n_views):
        nb, valid = tns[v]
        a, b, c = NR.e_norm_grad(sc, poses[v], intrs[v], nb.astype(np.float64), valid, sigma=sigma)
        acc[0] = acc[0] + W_NORM * np.asarray(a).reshape(acc[0].shape)
        acc[2] = acc[2] + W_NORM * np.asarray(b).reshape(acc[2].shape)
        gposes[v] = gposes[v] + W_NORM * c
        if face_sigma:
            gsig += W_NORM * _normal_sigma_grad(sc, poses[v], intrs[v], nb, valid, sigma)
    ref = acc + [np.concatenate(gposes)]
    names = ["grad_pos", "grad_col", "grad_opa", "grad_pose"]
    conds = cond + [None]
    if face_sigma:
        ref.append(gsig)
        names.append("grad_face_sigma")
        conds.append(None)
    for nm, a, b, cd in zip(names, got, ref, conds):
        ok, msg, _ = grad_close(a.reshape(-1), np.asarray(b, np.float64).reshape(-1), name=nm,
                                cond=None if cd is None else np.asarray(cd).reshape(-1))
        _say("  " + msg)
        assert ok, msg
    return rast


def _normal_sigma_grad(sc, pose, intr, nb, valid, sigma):
    """dE_norm/dsigma_m of the per-face exponents: the rasteriser backward of the soup with the
    world normals as colours and dE/dN_w = R^T dE/dN as the colour seed (the face normals do
    not depend on the exponents, nor does the rotation)."""
    ns = NR.normal_scene(sc)
    R = np.asarray(pose, np.float64).reshape(12)[:9].reshape(3, 3)
    m = np.asarray(valid, bool).reshape(-1)
    nbar = np.asarray(nb, np.float64).reshape(3, -1)
    gN = np.zeros_like(nbar)
    if m.any():
        gN[:, m] = -nbar[:, m] / m.sum()
    res = O.backward(ns, pose, intr, R.T @ gN, np.zeros(nbar.shape[1]), None, sigma=sigma, want_sigma=True)
    return np.asarray(res[4], np.float64)


@pytest.mark.parametrize("name,sigma,persp", [("single_64x48", 1.0, False), ("multi_view_mixed", 1.0, False),
                                              ("single_64x48", 0.5, False), ("tiny_ragged_50x37", 0.5, False),
                                              ("tiny_ragged_50x37", 2.0, False), ("long_tile_800", 1.0, False),
                                              ("tiny_ragged_50x37", 1.5, False), ("multi_view_mixed", 1.0, True),
                                              ("tiny_ragged_50x37", 2.0, True)])
def test_mapping_step_matches_oracle(name, sigma, persp):
    _say(f"[mapping] case={name} sigma={sigma} perspective={persp}")
    sc, poses, intrs = PAR._case(name)
    _run(sc, poses, intrs, 700, sigma=sigma, perspective=persp)


def test_mapping_step_views_of_different_sizes():
    _say("[mapping] three views of different sizes, perturbed poses")
    sc, intr = tiny_scene(33, n_faces=40, w=40, h=30, f=30.0)
    g = np.random.default_rng(33)
    poses = [left_perturb(IDENTITY, g.normal(scale=0.03, size=6)).astype(np.float32) for _ in range(3)]
    intrs = [intr, S.Intrinsics(33, 17, 30.0, 30.0, 16.0, 8.0), S.Intrinsics(20, 41, 28.0, 28.0, 10.0, 20.0)]
    _run(sc, poses, intrs, 710)


@pytest.mark.parametrize("name", ["tiny_ragged_50x37", "multi_view_mixed"])
def test_mapping_step_with_face_sigma(name):
    """Per-face exponents in [1, 2.5]; one view (per-wave staging) and three (cooperative)."""
    _say(f"[mapping] per-face exponents in [1, 2.5], case={name}")
    sc0, poses, intrs = PAR._case(name)
    g = np.random.default_rng(720)
    sc = S.Scene(sc0.pos, sc0.col, sc0.opa, None, g.uniform(1.0, 2.5, sc0.n_faces).astype(np.float32))
    _run(sc, poses, intrs, 720, face_sigma=True)


def test_mapping_step_room_20k_two_views():
    _say("[mapping] 20k-face room, two 96x72 views")
    sc = S.room_soup(34, 20_000, size_range=(0.01, 0.08))
    g = S.rng(35)
    poses = [S.random_room_pose(g), S.random_room_pose(g)]
    _run(sc, poses, [S.intrinsics_for(96, 72)] * 2, 730)


def test_one_binning_and_separate_normal_step_agree():
    """The mapping window with the normals as extra channels of one binning, and with the
    normal loss as a step of its own (a second binning of the normal-coloured soup): the same
    energy, so the same losses and gradients up to the order of the floating-point sums."""
    from paper_2605_31419_amd.window import MappingWindow
    _say("[mapping] one binning vs separate normal step, 4 views of a 20k-face room at 160x120")
    sc = S.room_soup(36, 20_000, size_range=(0.01, 0.08))
    dev = raster.DeviceScene.from_numpy(sc)
    g = S.rng(37)
    poses = raster.poses_tensor([S.random_room_pose(g) for _ in range(4)])
    intrs = [S.intrinsics_for(160, 120)] * 4
    P = 4 * 160 * 120
    gt = np.random.default_rng(38)
    tc = G.to_dev(gt.uniform(0, 1, 3 * P))
    td = G.to_dev(gt.uniform(0.5, 4.0, P))
    tn = raster.sensor_normals(td, intrs)
    res = []
    for fused in (True, False):
        win = MappingWindow(dev, intrs, w_ssim=W_SSIM, w_equi=1.2, w_norm=W_NORM, fused_mapping=fused)
        win.prepare(poses)
        grads = win.step(poses, tc, td, target_normals=tn)
        torch.cuda.synchronize()
        res.append(([x.cpu().numpy().astype(np.float64) for x in grads], win.loss.cpu().numpy(),
                    win.norm_loss.cpu().numpy(), float(win.equi_loss.cpu()[0])))
    (ga, la, na, ea), (gb, lb, nb_, eb) = res
    np.testing.assert_allclose(la, lb, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(na, nb_, rtol=1e-6, atol=1e-9)
    assert ea == eb
    for nm, a, b in zip(["grad_pos", "grad_col", "grad_opa", "grad_pose"], ga, gb):
        ok, msg, _ = grad_close(a, b, name=nm)
        _say("  " + msg)
        assert ok, msg


def test_indexed_meshes_are_refused():
    sc, intr = tiny_scene(36, n_faces=4)
    mesh = S.Scene(sc.pos, sc.col, sc.opa, np.arange(12, dtype=np.int32).reshape(4, 3))
    rast, p = G.make(mesh, [intr], [IDENTITY])
    rast.bin_and_sort(p)
    n = intr.width * intr.height
    z3, z1 = torch.zeros(3 * n, device="cuda"), torch.zeros(n, device="cuda")
    with pytest.raises(RuntimeError):
        rast.train_mapping(p, z3, z1, z3)


def test_mapping_step_replays_from_a_captured_graph():
    """The one-binning mapping step with E_equi (binning, forward with the normal channels, the
    D-SSIM stencils, the normal reduction, backward, chain, regulariser) captured in a HIP graph:
    the window's outputs are overwritten with NaN between replays, and every replay gives the
    eager step's losses and gradients (up to the order of the floating-point atomics)."""
    from paper_2605_31419_amd.window import MappingWindow
    _say("[mapping] graph capture, 3 views of a 20k-face room at 160x120")
    sc = S.room_soup(41, 20_000, size_range=(0.01, 0.08))
    dev = raster.DeviceScene.from_numpy(sc)
    g = S.rng(42)
    poses = raster.poses_tensor([S.random_room_pose(g) for _ in range(3)])
    intrs = [S.intrinsics_for(160, 120)] * 3
    P = 3 * 160 * 120
    gt = np.random.default_rng(43)
    tc = G.to_dev(gt.uniform(0, 1, 3 * P))
    td = G.to_dev(gt.uniform(0.5, 4.0, P))
    tn = raster.sensor_normals(td, intrs)
    win = MappingWindow(dev, intrs, w_ssim=W_SSIM, w_equi=1.2, w_norm=W_NORM)
    win.prepare(poses)
    eager = [x.clone() for x in win.step(poses, tc, td, target_normals=tn)]
    eloss = [win.loss.clone(), win.norm_loss.clone(), win.equi_loss.clone()]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        win.step(poses, tc, td, target_normals=tn)          # warm-up on the capture stream's kind
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        out = win.step(poses, tc, td, target_normals=tn)
    for rep in range(3):
        for x in list(out) + [win.loss, win.norm_loss, win.equi_loss, win.color]:
            x.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        from paper_2605_31419_amd import _lib
        _lib.check(win.rast.lib.tsr_check(raster._ptr(win.rast.ws), raster._stream(), None), "tsr_check")
        for a, b in zip([win.loss, win.norm_loss, win.equi_loss], eloss):
            np.testing.assert_allclose(a.cpu().numpy(), b.cpu().numpy(), rtol=1e-6, atol=1e-9)
        for nm, a, b in zip(["grad_pos", "grad_col", "grad_opa", "grad_pose"], out, eager):
            ok, msg, _ = grad_close(a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64), name=nm)
            if rep == 0:
                _say("  " + msg)
            assert ok, (rep, msg)


def test_mapping_step_on_an_empty_soup():
    """No faces: the image is the background (colour 0, depth 0), the normal map is 0, so every
    valid pixel adds 1 to the mean of 1 - N.N_bar (normal loss = w_norm), the photometric loss
    is the oracle's for a background render, and the pose gradient is 0."""
    from oracle import dssim as D
    _say("[mapping] empty soup")
    sc = S.Scene(np.zeros((3, 0), np.float32), np.zeros((3, 0), np.float32), np.zeros(0, np.float32))
    intr = S.intrinsics_for(64, 48)
    rast = raster.Rasterizer(raster.DeviceScene.from_numpy(sc), [intr])
    p = raster.poses_tensor([IDENTITY])
    rast.bin_and_sort(p)
    P = intr.width * intr.height
    g = np.random.default_rng(750)
    tc = g.uniform(0.1, 1, size=(3, P)).astype(np.float32)
    td = g.uniform(0.5, 4.0, size=P).astype(np.float32)
    nb, valid = _normal_targets(751, P)
    loss = torch.zeros(1, device="cuda")
    nloss = torch.zeros(1, device="cuda")
    nmap = torch.full((3 * P,), 7.0, device="cuda")
    out = rast.train_mapping(p, G.to_dev(tc), G.to_dev(td), G.to_dev(nb), w_ssim=W_SSIM, w_norm=W_NORM,
                             normal_map=nmap, loss=loss, loss_norm=nloss)
    torch.cuda.synchronize()
    oc, od, _ = O.render(sc, IDENTITY, intr)
    L, _, _ = O.l1_seeds(oc, od, tc, td, P)
    c3, t3 = np.asarray(oc, np.float64).reshape(3, intr.height, intr.width), tc.astype(np.float64).reshape(3, intr.height, intr.width)
    lref = L + W_SSIM * D.dssim(c3, t3)
    np.testing.assert_allclose(float(loss.cpu()[0]), lref, rtol=1e-5, atol=2e-5)
    np.testing.assert_allclose(float(nloss.cpu()[0]), W_NORM, rtol=1e-6)
    assert np.all(nmap.cpu().numpy() == 0.0)
    assert np.all(out[3].cpu().numpy() == 0.0)
