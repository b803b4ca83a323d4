"""GPU parity of the equilateral regulariser (Sec. 3.4, eq. 14) against the FP64 reference:
soups of 1 face to the 1M-face map, an indexed mesh with shared vertices, degenerate faces,
accumulate mode and the empty scene.  The kernel computes each face in FP64 and stores FP32
gradients, so gradients agree to FP32 rounding (1e-6 relative, floor 1e-7 of the largest
entry; indexed meshes add in atomic order); the loss, an FP64 sum, to 1e-6 relative."""
import numpy as np
import pytest
import torch

from oracle import equi as Q
from paper_2605_31419_amd import raster
from paper_2605_31419_amd import scenes as S
from tests.helpers import grad_close

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _dev(pos, faces=None):
    pos = np.ascontiguousarray(pos, np.float32)
    N = pos.shape[1]
    col = torch.zeros(3, N, device="cuda")
    opa = torch.zeros(N, device="cuda")
    f = None if faces is None else torch.as_tensor(np.asarray(faces, np.int32), device="cuda").contiguous()
    return raster.DeviceScene(torch.as_tensor(pos, device="cuda"), col, opa, f), pos


def _check(pos32, faces, loss, grad, weight=1.0):
    ref_l = Q.e_equi(pos32.astype(np.float64), faces)
    ref_g = weight * Q.e_equi_grad(pos32.astype(np.float64), faces)
    l = float(loss.cpu().numpy()[0])
    _say(f"  loss {l:.9g} ref {ref_l:.9g}")
    assert abs(l - ref_l) <= 1e-6 * abs(ref_l) + 1e-12
    ok, msg, _ = grad_close(grad.cpu().numpy(), ref_g, rel=1e-6, abs_frac=1e-7, name="grad_pos")
    _say("  " + msg)
    assert ok, msg


@pytest.mark.parametrize("M", [1, 255, 256, 1007])
def test_random_soups(M):
    pos = np.random.default_rng(M).normal(size=(3, 3 * M))
    sc, p32 = _dev(pos)
    loss, grad = raster.equilateral(sc, weight=1.2)
    torch.cuda.synchronize()
    _check(p32, None, loss, grad, weight=1.2)


def test_the_million_face_room_map():
    w = S.workload("track_1200x680_1M")
    sc = raster.DeviceScene.from_numpy(w.scene)
    loss, grad = raster.equilateral(sc)
    torch.cuda.synchronize()
    _check(np.asarray(w.scene.pos, np.float32), None, loss, grad)


def test_indexed_mesh_with_shared_vertices():
    g = np.random.default_rng(3)
    verts = g.normal(size=(3, 500))
    faces = np.array([g.choice(500, 3, replace=False) for _ in range(2000)])
    sc, p32 = _dev(verts, faces)
    loss, grad = raster.equilateral(sc)
    torch.cuda.synchronize()
    _check(p32, faces, loss, grad)


def test_degenerate_faces_and_unused_vertices():
    g = np.random.default_rng(4)
    pos = g.normal(size=(3, 3 * 40 + 5))                 # 5 trailing vertices belong to no face
    pos[:, 3] = pos[:, 4]                                # face 1: two equal corners
    pos[:, 30:33] = pos[:, 30:31]                        # face 10: a point
    sc, p32 = _dev(pos)
    sc.n_faces = 40
    grad = torch.full((3, pos.shape[1]), float("nan"), device="cuda")
    loss, grad = raster.equilateral(sc, grad=grad)
    torch.cuda.synchronize()
    gn = grad.cpu().numpy()
    assert np.all(gn[:, 3:6] == 0) and np.all(gn[:, 30:33] == 0) and np.all(gn[:, 120:] == 0)
    _check(p32[:, :120], None, loss, grad[:, :120])


def test_accumulate_adds():
    pos = np.random.default_rng(5).normal(size=(3, 300))
    sc, p32 = _dev(pos)
    _, g1 = raster.equilateral(sc)
    base = torch.as_tensor(np.random.default_rng(6).normal(size=(3, 300)).astype(np.float32), device="cuda")
    acc = base.clone()
    raster.equilateral(sc, weight=0.5, grad=acc, accumulate=True)
    torch.cuda.synchronize()
    np.testing.assert_allclose(acc.cpu().numpy(), base.cpu().numpy() + 0.5 * g1.cpu().numpy(), rtol=0, atol=1e-6)


def test_empty_scene():
    sc, _ = _dev(np.zeros((3, 0)))
    loss, grad = raster.equilateral(sc)
    torch.cuda.synchronize()
    assert float(loss.cpu().numpy()[0]) == 0.0 and grad.numel() == 0
