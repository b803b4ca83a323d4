"""GPU parity of the per-face window exponent (Sec. 3.2 after eq. 3: Triangle Splatting's
learnable per-triangle sigma), through the C ABI, against the FP64 oracle with the same
exponents: forward images, the backward's four gradients plus dL/dsigma_m, the fused L1
step, the photometric step with D-SSIM, face statistics, the autograd Function, and the
reduction to the global path when every face has the same exponent.

Exponents below 1 have the steep-edge band of the sigma < 1 window; as for the global path,
upstream gradients are zeroed on both sides at pixels within |rho| < 1e-3 of a face edge
(steps whose seeds the kernels form themselves use exponents in [1, 2.5])."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2605_31419_amd import raster
from paper_2605_31419_amd import scenes as S
from tests import gpu_util as G
from tests import test_gpu_parity as PAR
from tests.helpers import grad_close

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4


def _say(*a):
    print(*a, flush=True)


def _case(name, lo, hi, seed=5):
    sc, poses, intrs = PAR._case(name)
    g = np.random.default_rng(seed)
    fs = g.uniform(lo, hi, size=sc.n_faces).astype(np.float32)
    return S.Scene(sc.pos, sc.col, sc.opa, sc.faces, fs), poses, intrs


def _make(sc, intrs, poses, sigma=1.0):
    return G.make(sc, intrs, poses, sigma=sigma)


def _oracle_views(sc, poses, intrs, gcs, gds, gts):
    """Oracle gradients summed over the views (pose gradients concatenated per view):
    [pos, col, opa, pose, dL/dsigma], and the conditioning of each element (sums of absolute
    per-pixel terms; None for the pose)."""
    acc = [0.0] * 4
    cond = [0.0] * 4
    gposes = []
    for v in range(len(poses)):
        gp, gc, go, gpose, gs, ab = O.backward(sc, poses[v], intrs[v], gcs[v], gds[v],
                                               None if gts is None else gts[v], want_sigma=True, with_abs=True)
        acc = [acc[0] + gp, acc[1] + gc, acc[2] + go, acc[3] + gs]
        cond = [c + x for c, x in zip(cond, ab)]
        gposes.append(gpose)
    return [acc[0], acc[1], acc[2], np.concatenate(gposes), acc[3]], [cond[0], cond[1], cond[2], None, cond[3]]


@pytest.mark.parametrize("name", ["single_64x48", "tiny_ragged_50x37", "multi_view_mixed", "long_tile_800",
                                  "huge_faces_640x480"])
def test_forward_with_face_sigma(name):
    _say(f"[face sigma forward] case={name}")
    sc, poses, intrs = _case(name, 0.4, 2.5)
    rast, p = _make(sc, intrs, poses, sigma=1.0)       # the global value is ignored
    c, d, t = G.render(rast, p)
    cs, ds, ts = G.per_view(rast, c, 3), G.per_view(rast, d, 1), G.per_view(rast, t, 1)
    for v in range(len(poses)):
        oc, od, ot = O.render(sc, poses[v], intrs[v])
        err = max(np.abs(cs[v] - oc).max(), np.abs(ds[v] - od).max(), np.abs(ts[v] - ot).max())
        _say(f"  view {v}: max abs err {err:.3e}")
        assert err <= IMG_TOL


@pytest.mark.parametrize("name", ["single_64x48", "tiny_ragged_50x37", "multi_view_mixed", "long_tile_800",
                                  "huge_faces_640x480"])
def test_backward_with_face_sigma(name):
    _say(f"[face sigma backward] case={name}")
    sc, poses, intrs = _case(name, 0.4, 2.5)
    rast, p = _make(sc, intrs, poses)
    P = rast.total_pixels
    g = np.random.default_rng(43)
    gc = g.normal(size=3 * P).astype(np.float32)
    gd = g.normal(size=P).astype(np.float32)
    gt = g.normal(size=P).astype(np.float32)
    masks = PAR._steep_masks(sc, poses, intrs, 0.5)
    for a, ch in ((gc, 3), (gd, 1), (gt, 1)):
        PAR._apply_masks(a, masks, ch)
    _say(f"  steep-edge and ridge pixels masked on both sides: {sum(int(m.sum()) for m in masks)} of {P}")
    rast.bin_and_sort(p)
    rast.forward(p)
    out = rast.backward(p, G.to_dev(gc), G.to_dev(gd), G.to_dev(gt))
    torch.cuda.synchronize()
    got = [x.cpu().numpy().astype(np.float64) for x in out] + [rast.grad_face_sigma.cpu().numpy().astype(np.float64)]
    gcs, gds, gts = G.per_view(rast, gc, 3), G.per_view(rast, gd, 1), G.per_view(rast, gt, 1)
    ref, conds = _oracle_views(sc, poses, intrs, gcs, gds, gts)
    for nm, a, b, cond in zip(["grad_pos", "grad_col", "grad_opa", "grad_pose", "grad_face_sigma"], got, ref, conds):
        ok, msg, _ = grad_close(a, b, name=nm, cond=cond)
        _say("  " + msg)
        assert ok, msg


@pytest.mark.parametrize("name", ["single_64x48", "multi_view_mixed", "long_tile_800"])
def test_train_l1_with_face_sigma(name):
    _say(f"[face sigma train_l1] case={name}")
    sc, poses, intrs = _case(name, 1.0, 2.5)
    rast, p = _make(sc, intrs, poses)
    tcs, tds, gseeds, lossref = [], [], [], []
    for v in range(len(poses)):
        oc, od, ot = O.render(sc, poses[v], intrs[v])
        tc, td, _ = PAR._nudged_targets(oc, od, 200 + v, None)
        L, gcv, gdv = O.l1_seeds(oc, od, tc, td, intrs[v].width * intrs[v].height)
        tcs.append(tc); tds.append(td); gseeds.append((gcv, gdv)); lossref.append(L)
    rast.bin_and_sort(p)
    loss = torch.zeros(len(poses), device="cuda")
    out = rast.train_l1(p, G.to_dev(np.concatenate([t.reshape(-1) for t in tcs])),
                        G.to_dev(np.concatenate([t.reshape(-1) for t in tds])), loss=loss)
    torch.cuda.synchronize()
    np.testing.assert_allclose(loss.cpu().numpy(), lossref, rtol=1e-5)
    got = [x.cpu().numpy().astype(np.float64) for x in out] + [rast.grad_face_sigma.cpu().numpy().astype(np.float64)]
    acc, conds = _oracle_views(sc, poses, intrs, [s_[0] for s_ in gseeds], [s_[1] for s_ in gseeds], None)
    for nm, a, b, cond in zip(["grad_pos", "grad_col", "grad_opa", "grad_pose", "grad_face_sigma"], got, acc, conds):
        ok, msg, _ = grad_close(a, b, name=nm, cond=cond)
        _say("  " + msg)
        assert ok, msg


def test_photometric_step_with_face_sigma():
    """Eqs. 8 and 10 with the D-SSIM term: the oracle's L1 + 0.2 D-SSIM seeds of the oracle
    render pushed through the oracle backward, including dL/dsigma_m."""
    from oracle import dssim as D
    sc, poses, intrs = _case("tiny_ragged_50x37", 1.0, 2.5)
    rast, p = _make(sc, intrs, poses)
    W, H = intrs[0].width, intrs[0].height
    oc, od, ot = O.render(sc, poses[0], intrs[0])
    tc, td, _ = PAR._nudged_targets(oc, od, 301, None)
    L, gcv, gdv = O.l1_seeds(oc, od, tc, td, W * H)
    c3, t3 = np.asarray(oc).reshape(3, H, W), tc.astype(np.float64).reshape(3, H, W)
    gcv = gcv + 0.2 * D.dssim_grad(c3, t3).reshape(gcv.shape)
    rast.bin_and_sort(p)
    P = rast.total_pixels
    out = rast.train_photometric(p, G.to_dev(tc), G.to_dev(td), w_ssim=0.2, color=torch.empty(3 * P, device="cuda"),
                                 depth=torch.empty(P, device="cuda"))
    torch.cuda.synchronize()
    got = [x.cpu().numpy().astype(np.float64) for x in out] + [rast.grad_face_sigma.cpu().numpy().astype(np.float64)]
    ref = O.backward(sc, poses[0], intrs[0], gcv, gdv, None, want_sigma=True)
    for nm, a, b in zip(["grad_pos", "grad_col", "grad_opa", "grad_pose", "grad_face_sigma"], got, ref):
        ok, msg, _ = grad_close(a, b, name=nm)
        _say("  " + msg)
        assert ok, msg


def test_face_stats_with_face_sigma():
    from tests import test_gpu_stats as ST
    sc0, intr = ST.tiny_scene(16, n_faces=40, w=48, h=36, f=36.0)
    g = np.random.default_rng(16)
    sc = S.Scene(sc0.pos, sc0.col, sc0.opa, None, g.uniform(0.4, 2.5, sc0.n_faces).astype(np.float32))
    _, _, area, cov, vis = ST._gpu_stats(sc, [intr], [ST.IDENTITY], t_min=0.3)
    ST._check_view(sc, ST.IDENTITY, intr, area, cov, vis, 0.3)


def test_uniform_face_sigma_equals_the_global_exponent():
    """Every face at sigma = 0.75: the per-face kernels evaluate the same instructions as the
    global generic-exponent kernels, so the images are bitwise equal and the gradients equal up
    to the order of the floating-point atomics."""
    sc, poses, intrs = PAR._case("tiny_ragged_50x37")
    fs = S.Scene(sc.pos, sc.col, sc.opa, None, np.full(sc.n_faces, 0.75, np.float32))
    ra, pa = _make(sc, intrs, poses, sigma=0.75)
    rb, pb = _make(fs, intrs, poses, sigma=1.0)
    P = ra.total_pixels
    g = np.random.default_rng(3)
    gc, gd = G.to_dev(g.normal(size=3 * P)), G.to_dev(g.normal(size=P))
    outs = []
    for r, p in ((ra, pa), (rb, pb)):
        r.bin_and_sort(p)
        img = r.forward(p)
        grads = r.backward(p, gc, gd, None)
        torch.cuda.synchronize()
        outs.append(([x.cpu().numpy() for x in img], [x.cpu().numpy() for x in grads]))
    for a, b in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, b)
    for a, b in zip(outs[0][1], outs[1][1]):
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-6 * np.abs(a).max())


def test_autograd_returns_the_face_sigma_gradient():
    sc, poses, intrs = _case("single_64x48", 1.0, 2.5)
    dev = raster.DeviceScene.from_numpy(sc)
    dev.face_sigma.requires_grad_(True)
    rast = raster.Rasterizer(dev, intrs)
    pt = raster.poses_tensor(poses)
    rast.fit(pt)
    color, depth, trans = raster.rasterize(rast, pt)
    P = rast.total_pixels
    g = np.random.default_rng(8)
    wc, wd = g.normal(size=3 * P), g.normal(size=P)
    loss = (torch.as_tensor(wc, dtype=torch.float32, device="cuda") * color).sum() + \
           (torch.as_tensor(wd, dtype=torch.float32, device="cuda") * depth).sum()
    loss.backward()
    ref = O.backward(sc, poses[0], intrs[0], wc.astype(np.float32).astype(np.float64).reshape(3, P),
                     wd.astype(np.float32).astype(np.float64), None, want_sigma=True)[4]
    ok, msg, _ = grad_close(dev.face_sigma.grad.cpu().numpy(), ref, name="face_sigma.grad")
    _say("  " + msg)
    assert ok, msg
