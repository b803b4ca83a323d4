"""GPU parity of the perspective-correct variant (colour with perspective-correct barycentrics,
depth of the face's plane along the ray) against the FP64 oracle with the same rule: forward
images, the backward's gradients, the fused L1 step and the photometric step, at several window
exponents, one and several views; and the refusal to combine it with per-face exponents."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2605_31419_amd import _lib, raster
from paper_2605_31419_amd import scenes as S
from tests import gpu_util as G
from tests import test_gpu_parity as PAR
from tests.helpers import grad_close

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4


def _say(*a):
    print(*a, flush=True)


def _make(sc, intrs, poses, sigma=1.0):
    d = raster.DeviceScene.from_numpy(sc)
    rast = raster.Rasterizer(d, intrs, raster.Params(sigma=sigma, perspective=True))
    p = raster.poses_tensor(poses)
    rast.fit(p)
    return rast, p


@pytest.mark.parametrize("name", ["single_64x48", "tiny_ragged_50x37", "multi_view_mixed", "huge_faces_640x480",
                                  "long_tile_800", "max_views_32"])
@pytest.mark.parametrize("sigma", [1.0, 0.5])
def test_forward_perspective(name, sigma):
    _say(f"[perspective forward] case={name} sigma={sigma}")
    sc, poses, intrs = PAR._case(name)
    rast, p = _make(sc, intrs, poses, sigma)
    c, d, t = G.render(rast, p)
    cs, ds, ts = G.per_view(rast, c, 3), G.per_view(rast, d, 1), G.per_view(rast, t, 1)
    for v in range(len(poses)):
        oc, od, ot = O.render(sc, poses[v], intrs[v], sigma=sigma, perspective=True)
        err = max(np.abs(cs[v] - oc).max(), np.abs(ds[v] - od).max(), np.abs(ts[v] - ot).max())
        _say(f"  view {v}: max abs err {err:.3e}")
        assert err <= IMG_TOL


@pytest.mark.parametrize("name", ["single_64x48", "tiny_ragged_50x37", "multi_view_mixed", "huge_faces_640x480",
                                  "long_tile_800"])
@pytest.mark.parametrize("sigma", [1.0, 0.5, 2.0])
def test_backward_perspective(name, sigma):
    _say(f"[perspective backward] case={name} sigma={sigma}")
    sc, poses, intrs = PAR._case(name)
    rast, p = _make(sc, intrs, poses, sigma)
    P = rast.total_pixels
    g = np.random.default_rng(42)
    gc = g.normal(size=3 * P).astype(np.float32)
    gd = g.normal(size=P).astype(np.float32)
    gt = g.normal(size=P).astype(np.float32)
    masks = PAR._steep_masks(sc, poses, intrs, sigma)
    for a, ch in ((gc, 3), (gd, 1), (gt, 1)):
        PAR._apply_masks(a, masks, ch)
    rast.bin_and_sort(p)
    rast.forward(p)
    out = rast.backward(p, G.to_dev(gc), G.to_dev(gd), G.to_dev(gt))
    torch.cuda.synchronize()
    got = [x.cpu().numpy().astype(np.float64) for x in out]
    gcs, gds, gts = G.per_view(rast, gc, 3), G.per_view(rast, gd, 1), G.per_view(rast, gt, 1)
    acc, cond = [0.0] * 3, [0.0] * 3
    gposes = []
    for v in range(len(poses)):
        gp, gcol, go, gpose, ab = O.backward(sc, poses[v], intrs[v], gcs[v], gds[v], gts[v], sigma=sigma,
                                             with_abs=True, perspective=True)
        acc = [acc[0] + gp, acc[1] + gcol, acc[2] + go]
        cond = [c + x for c, x in zip(cond, ab)]
        gposes.append(gpose)
    ref = acc + [np.concatenate(gposes)]
    for nm, a, b, cd in zip(["grad_pos", "grad_col", "grad_opa", "grad_pose"], got, ref, cond + [None]):
        ok, msg, _ = grad_close(a, b, name=nm, cond=cd)
        _say("  " + msg)
        assert ok, msg


@pytest.mark.parametrize("name", ["single_64x48", "multi_view_mixed", "long_tile_800"])
def test_train_l1_perspective(name):
    _say(f"[perspective train_l1] case={name}")
    sc, poses, intrs = PAR._case(name)
    rast, p = _make(sc, intrs, poses)
    tcs, tds, seeds, lossref = [], [], [], []
    for v in range(len(poses)):
        oc, od, ot = O.render(sc, poses[v], intrs[v], perspective=True)
        tc, td, _ = PAR._nudged_targets(oc, od, 400 + v, None)
        L, gcv, gdv = O.l1_seeds(oc, od, tc, td, intrs[v].width * intrs[v].height)
        tcs.append(tc); tds.append(td); seeds.append((gcv, gdv)); lossref.append(L)
    rast.bin_and_sort(p)
    loss = torch.zeros(len(poses), device="cuda")
    out = rast.train_l1(p, G.to_dev(np.concatenate([t.reshape(-1) for t in tcs])),
                        G.to_dev(np.concatenate([t.reshape(-1) for t in tds])), loss=loss)
    torch.cuda.synchronize()
    np.testing.assert_allclose(loss.cpu().numpy(), lossref, rtol=1e-5)
    got = [x.cpu().numpy().astype(np.float64) for x in out]
    acc = [0.0] * 3
    gposes = []
    for v in range(len(poses)):
        gp, gcol, go, gpose = O.backward(sc, poses[v], intrs[v], seeds[v][0], seeds[v][1], None, perspective=True)
        acc = [acc[0] + gp, acc[1] + gcol, acc[2] + go]
        gposes.append(gpose)
    for nm, a, b in zip(["grad_pos", "grad_col", "grad_opa", "grad_pose"], got, acc + [np.concatenate(gposes)]):
        ok, msg, _ = grad_close(a, b, name=nm)
        _say("  " + msg)
        assert ok, msg


def test_photometric_step_perspective():
    from oracle import dssim as D
    sc, poses, intrs = PAR._case("tiny_ragged_50x37")
    rast, p = _make(sc, intrs, poses)
    W, H = intrs[0].width, intrs[0].height
    oc, od, ot = O.render(sc, poses[0], intrs[0], perspective=True)
    tc, td, _ = PAR._nudged_targets(oc, od, 401, None)
    L, gcv, gdv = O.l1_seeds(oc, od, tc, td, W * H)
    gcv = gcv + 0.2 * D.dssim_grad(np.asarray(oc).reshape(3, H, W), tc.astype(np.float64).reshape(3, H, W)).reshape(gcv.shape)
    rast.bin_and_sort(p)
    P = rast.total_pixels
    out = rast.train_photometric(p, G.to_dev(tc), G.to_dev(td), w_ssim=0.2, color=torch.empty(3 * P, device="cuda"),
                                 depth=torch.empty(P, device="cuda"))
    torch.cuda.synchronize()
    got = [x.cpu().numpy().astype(np.float64) for x in out]
    ref = O.backward(sc, poses[0], intrs[0], gcv, gdv, None, perspective=True)
    for nm, a, b in zip(["grad_pos", "grad_col", "grad_opa", "grad_pose"], got, ref):
        ok, msg, _ = grad_close(a, b, name=nm)
        _say("  " + msg)
        assert ok, msg


def test_perspective_with_face_sigma_is_refused():
    sc, poses, intrs = PAR._case("single_64x48")
    sc = S.Scene(sc.pos, sc.col, sc.opa, None, np.ones(sc.n_faces, np.float32))
    d = raster.DeviceScene.from_numpy(sc)
    with pytest.raises(_lib.TsrError):
        rast = raster.Rasterizer(d, intrs, raster.Params(perspective=True))
        rast.fit(raster.poses_tensor(poses))
