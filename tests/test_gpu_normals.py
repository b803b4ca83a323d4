"""GPU parity of the normal supervision of mapping (Sec. 3.4) against the FP64 reference:
sensor normals from depth (planes, depth with holes, several views of ragged sizes), and the
normal-loss step (rendered normal map, loss, position / opacity / pose gradients) on tiny
scenes, several views and a 20k-face room.  Tolerances: sensor normals within 1e-6 (FP64 on
both sides, FP32 output), validity identical; the normal map within 1e-5 (as images); the
loss within 1e-5 relative; gradients as the rasterizer's backward (1e-3 relative)."""
import numpy as np
import pytest
import torch

from oracle import normals as NR
from paper_2605_31419_amd import raster
from paper_2605_31419_amd import scenes as S
from tests import gpu_util as G
from tests.helpers import IDENTITY, grad_close, left_perturb, tiny_scene

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _depths(seed, intrs):
    g = np.random.default_rng(seed)
    out = []
    for k, it in enumerate(intrs):
        v, u = np.mgrid[0:it.height, 0:it.width].astype(np.float64)
        n = g.normal(size=3)
        n[2] = abs(n[2]) + 1.0
        n /= np.linalg.norm(n)
        ray = np.stack([(u - it.cx) / it.fx, (v - it.cy) / it.fy, np.ones_like(u)])
        d = 2.0 / np.tensordot(n, ray, axes=1)
        d += 0.01 * np.sin(0.3 * u + 0.2 * v + k)            # a curved surface
        d[g.uniform(size=d.shape) < 0.05] = 0.0              # holes
        out.append(d.astype(np.float32))
    return out


def test_sensor_normals_match_the_reference():
    intrs = [S.intrinsics_for(64, 48), S.intrinsics_for(37, 23), S.Intrinsics(3, 5, 4.0, 4.0, 1.0, 2.0),
             S.intrinsics_for(1200, 680)]
    ds = _depths(1, intrs)
    dev = torch.as_tensor(np.concatenate([d.reshape(-1) for d in ds]), device="cuda")
    got = raster.sensor_normals(dev, intrs).cpu().numpy()
    off = 0
    for it, d in zip(intrs, ds):
        P = it.width * it.height
        g = got[3 * off:3 * (off + P)].reshape(3, it.height, it.width)
        ref, valid = NR.sensor_normals(d, it)
        gv = np.any(g != 0, axis=0)
        assert np.array_equal(gv, valid), (it, int((gv != valid).sum()))
        err = np.abs(g - ref).max()
        _say(f"  {it.width}x{it.height}: valid {int(valid.sum())} / {P}, max err {err:.2e}")
        assert err <= 1e-6
        off += P


def _targets(seed, n_pix, frac_valid=0.8):
    g = np.random.default_rng(seed)
    nb = g.normal(size=(3, n_pix))
    nb /= np.linalg.norm(nb, axis=0)
    valid = g.uniform(size=n_pix) < frac_valid
    nb[:, ~valid] = 0.0
    return nb.astype(np.float32), valid


def _run(sc, intrs, poses, seed, w_norm=0.05, sigma=1.0):
    rast, p = G.make(sc, intrs, poses, sigma=sigma)
    tgts = [_targets(seed + v, it.width * it.height) for v, it in enumerate(intrs)]
    tdev = torch.as_tensor(np.concatenate([t.reshape(-1) for t, _ in tgts]), device="cuda")
    P = rast.total_pixels
    nmap = torch.empty(3 * P, device="cuda")
    loss = torch.empty(len(intrs), device="cuda")
    gp, go, gpose = rast.train_normal(p, tdev, w_norm=w_norm, normal_map=nmap, loss=loss)
    torch.cuda.synchronize()
    got = [gp.cpu().numpy(), go.cpu().numpy(), gpose.cpu().numpy()]
    ref = [np.zeros((3, sc.n_vertices)), np.zeros(sc.n_vertices), []]
    nm = nmap.cpu().numpy()
    off = 0
    for v, (it, (nb, valid)) in enumerate(zip(intrs, tgts)):
        Pv = it.width * it.height
        nb64 = nb.astype(np.float64)
        lref = w_norm * NR.e_norm(sc, poses[v], it, nb64, valid, sigma=sigma)
        a, b, c = NR.e_norm_grad(sc, poses[v], it, nb64, valid, sigma=sigma)
        ref[0] += w_norm * a
        ref[1] += w_norm * b
        ref[2].append(w_norm * c)
        nref = NR.render_normals(sc, poses[v], it, sigma=sigma)
        err = np.abs(nm[3 * off:3 * (off + Pv)].reshape(3, Pv) - nref).max()
        _say(f"  view {v}: loss {float(loss[v]):.7f} ref {lref:.7f}, normal map err {err:.2e}")
        assert err <= 1e-5
        assert abs(float(loss[v]) - lref) <= 1e-5 * abs(lref) + 1e-9
        off += Pv
    ref[2] = np.concatenate(ref[2])
    for nm_, a, b in zip(["grad_pos", "grad_opa", "grad_pose"], got, ref):
        ok, msg, _ = grad_close(a, b, name=nm_)
        _say("  " + msg)
        assert ok, msg
    return rast


@pytest.mark.parametrize("seed,sigma", [(31, 1.0), (32, 1.0), (33, 0.5), (34, 2.0)])
def test_normal_step_tiny(seed, sigma):
    sc, intr = tiny_scene(seed, n_faces=30, w=48, h=36, f=36.0)
    pose = left_perturb(IDENTITY, np.random.default_rng(seed).normal(scale=0.03, size=6)).astype(np.float32)
    _run(sc, [intr], [pose], seed, sigma=sigma)


def test_normal_step_views_of_different_sizes():
    sc, intr = tiny_scene(33, n_faces=40, w=40, h=30, f=30.0)
    g = np.random.default_rng(33)
    poses = [left_perturb(IDENTITY, g.normal(scale=0.03, size=6)).astype(np.float32) for _ in range(3)]
    intrs = [intr, S.Intrinsics(33, 17, 30.0, 30.0, 16.0, 8.0), S.Intrinsics(20, 41, 28.0, 28.0, 10.0, 20.0)]
    _run(sc, intrs, poses, 40)


def test_normal_step_room_20k():
    sc = S.room_soup(34, 20_000, size_range=(0.01, 0.08))
    g = S.rng(35)
    pose = S.random_room_pose(g)
    _run(sc, [S.intrinsics_for(96, 72)], [pose], 50)


def test_indexed_meshes_are_refused():
    from paper_2605_31419_amd import _lib
    sc, intr = tiny_scene(36, n_faces=4)
    faces = np.arange(12, dtype=np.int32).reshape(4, 3)
    mesh = S.Scene(sc.pos, sc.col, sc.opa, faces)
    rast, p = G.make(mesh, [intr], [IDENTITY])
    tgt = torch.zeros(3 * intr.width * intr.height, device="cuda")
    with pytest.raises(RuntimeError):
        rast.train_normal(p, tgt)


def test_accumulate_adds_and_leaves_extra_vertices_alone():
    """accumulate adds the gradients to the buffers; a soup's vertices past 3M (no face uses
    them) keep their values."""
    sc, intr = tiny_scene(37, n_faces=30, w=48, h=36, f=36.0)
    extra = 5
    g = np.random.default_rng(37)
    pos = np.concatenate([sc.pos, g.normal(size=(3, extra)).astype(np.float32)], axis=1)
    col = np.concatenate([sc.col, np.zeros((3, extra), np.float32)], axis=1)
    opa = np.concatenate([sc.opa, np.full(extra, 0.5, np.float32)])
    dev = raster.DeviceScene(torch.as_tensor(pos, device="cuda"), torch.as_tensor(col, device="cuda"),
                             torch.as_tensor(opa, device="cuda"))
    dev.n_faces = 30
    rast = raster.Rasterizer(dev, [intr])
    p = raster.poses_tensor([IDENTITY])
    rast.fit(p)
    nb, _ = _targets(38, intr.width * intr.height)
    t = torch.as_tensor(nb.reshape(-1), device="cuda")
    ref = [x.clone() for x in rast.train_normal(p, t, w_norm=0.05)]
    N = pos.shape[1]
    gp = torch.ones(3 * N, device="cuda")
    go = torch.ones(N, device="cuda")
    gpose = torch.ones(6, device="cuda")
    rast.train_normal(p, t, w_norm=0.05, out=(gp, go, gpose), accumulate=True)
    torch.cuda.synchronize()
    gpn, gon = gp.cpu().numpy().reshape(3, N), go.cpu().numpy()
    assert np.all(gpn[:, 90:] == 1.0) and np.all(gon[90:] == 1.0)
    np.testing.assert_allclose(gpn[:, :90], 1.0 + ref[0].cpu().numpy().reshape(3, N)[:, :90], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(gon[:90], 1.0 + ref[1].cpu().numpy()[:90], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(gpose.cpu().numpy(), 1.0 + ref[2].cpu().numpy(), rtol=1e-6, atol=1e-6)


def test_sensor_normals_of_32_views():
    g = np.random.default_rng(39)
    intrs = [S.Intrinsics(int(w), int(h), 30.0, 30.0, (int(w) - 1) / 2, (int(h) - 1) / 2)
             for w, h in g.integers(1, 40, size=(32, 2))]
    ds = _depths(40, intrs)
    got = raster.sensor_normals(torch.as_tensor(np.concatenate([d.reshape(-1) for d in ds]), device="cuda"),
                                intrs).cpu().numpy()
    off = 0
    for it, d in zip(intrs, ds):
        P = it.width * it.height
        ref, valid = NR.sensor_normals(d, it)
        gv = got[3 * off:3 * (off + P)].reshape(3, it.height, it.width)
        assert np.array_equal(np.any(gv != 0, axis=0), valid)
        assert np.abs(gv - ref).max() <= 1e-6
        off += P
