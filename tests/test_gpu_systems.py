"""GPU tests of the systems built around the kernels: the autograd Function, the batched
mapping window with autotuned schedules, the captured tracking loop, and the serving loop."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2605_31419_amd import autotune, raster
from paper_2605_31419_amd import scenes as S
from paper_2605_31419_amd.serve import GpuExecutor, Request, Server
from paper_2605_31419_amd.track import Tracker
from paper_2605_31419_amd.window import MappingWindow
from tests import gpu_util as G
from tests.helpers import IDENTITY, grad_close, left_perturb, tiny_scene

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------------------- autograd

def test_autograd_function_matches_oracle():
    sc, intr = tiny_scene(21, n_faces=40, w=48, h=36, f=36.0)
    pose = left_perturb(IDENTITY, np.array([0.01, -0.02, 0.0, 0.02, 0.01, -0.01])).astype(np.float32)
    dev = raster.DeviceScene.from_numpy(sc)
    for t in (dev.pos, dev.col, dev.opa):
        t.requires_grad_(True)
    rast = raster.Rasterizer(dev, [intr])
    poses = raster.poses_tensor([pose])
    rast.fit(poses)
    tau = torch.zeros(1, 6, device="cuda", requires_grad=True)
    color, depth, trans = raster.rasterize(rast, poses, tau)
    P = intr.width * intr.height
    g = np.random.default_rng(3)
    wc, wd, wt = (torch.as_tensor(g.normal(size=n).astype(np.float32), device="cuda") for n in (3 * P, P, P))
    loss = (wc * color).sum() + (wd * depth).sum() + (wt * trans).sum()
    loss.backward()
    ref = O.backward(sc, pose, intr, wc.cpu().numpy().reshape(3, P), wd.cpu().numpy(), wt.cpu().numpy())
    got = [dev.pos.grad, dev.col.grad, dev.opa.grad, tau.grad.reshape(-1)]
    for nm, a, b in zip(["pos", "col", "opa", "tau"], got, ref):
        ok, msg, _ = grad_close(a.detach().cpu().numpy(), b, name=nm)
        _say("  " + msg)
        assert ok, msg


def _numeric_left_jacobian(tau, h=1e-6):
    """J_l(tau) by central differences of Log(Exp(tau + h e_k) Exp(tau)^-1) (scipy's matrix
    exponential and logarithm), columns in (rho, theta) order."""
    import scipy.linalg

    from tests.helpers import se3_exp
    inv0 = np.linalg.inv(se3_exp(tau))
    J = np.zeros((6, 6))
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        d = (scipy.linalg.logm(se3_exp(tau + e) @ inv0) - scipy.linalg.logm(se3_exp(tau - e) @ inv0)).real / (2 * h)
        J[:, k] = [d[0, 3], d[1, 3], d[2, 3], d[2, 1], d[0, 2], d[1, 0]]
    return J


def test_pose_compose_matches_matrix_exponential():
    """tsr_pose_compose against scipy's matrix exponential of the se(3) generator (eq. 6), for
    zero, tiny, moderate and large rotations."""
    g = np.random.default_rng(5)
    poses = np.stack([left_perturb(IDENTITY, g.normal(scale=0.4, size=6)).astype(np.float32) for _ in range(5)])
    taus = np.stack([np.zeros(6), np.full(6, 1e-7), g.normal(scale=0.05, size=6),
                     np.concatenate([g.normal(scale=0.3, size=3), g.normal(scale=0.4, size=3)]),
                     np.array([0.2, -0.1, 0.3, 1.5, -1.7, 0.9])]).astype(np.float32)
    out = raster.compose_poses(torch.as_tensor(taus, device="cuda"), torch.as_tensor(poses, device="cuda"))
    got = out.cpu().numpy().astype(np.float64)
    ref = np.stack([left_perturb(poses[i].astype(np.float64), taus[i].astype(np.float64)) for i in range(5)])
    err = np.abs(got - ref).max()
    _say(f"  compose: max abs err {err:.2e}")
    assert err <= 2e-6


def test_tau_gradient_is_the_left_jacobian_transpose():
    """tsr_pose_tau_grad = J_l(tau)^T g with J_l from scipy's matrix logarithm (central
    differences), for tau from zero to a 2.6 rad rotation."""
    g = np.random.default_rng(6)
    taus = np.stack([np.zeros(6), g.normal(scale=0.05, size=6), np.array([0.3, -0.2, 0.1, 1.2, 2.0, -1.0])])
    grads = g.normal(size=(3, 6))
    out = raster.tau_gradient(torch.as_tensor(taus, dtype=torch.float32, device="cuda"),
                              torch.as_tensor(grads, dtype=torch.float32, device="cuda")).cpu().numpy()
    for i in range(3):
        t32 = taus[i].astype(np.float32).astype(np.float64)
        ref = _numeric_left_jacobian(t32).T @ grads[i].astype(np.float32).astype(np.float64)
        ok, msg, _ = grad_close(out[i], ref, rel=1e-5, abs_frac=1e-6, name=f"tau {i}")
        _say("  " + msg)
        assert ok, msg


def test_autograd_pose_gradient_at_nonzero_tau():
    """rasterize() at tau != 0: the scene is rendered at Exp(tau) T and tau.grad is dL/dtau --
    checked against the oracle's left-perturbation gradient at that pose mapped by the numeric
    J_l(tau)^T, which is itself checked against FP64 central differences of the oracle loss in
    tau."""
    sc, intr = tiny_scene(21, n_faces=40, w=48, h=36, f=36.0)
    pose = left_perturb(IDENTITY, np.array([0.01, -0.02, 0.0, 0.02, 0.01, -0.01])).astype(np.float32)
    tau0 = np.array([0.03, -0.02, 0.01, 0.05, -0.04, 0.03], np.float32)
    dev = raster.DeviceScene.from_numpy(sc)
    rast = raster.Rasterizer(dev, [intr])
    poses = raster.poses_tensor([pose])
    rast.fit(raster.compose_poses(torch.as_tensor(tau0[None], device="cuda"), poses))
    tau = torch.as_tensor(tau0[None], device="cuda").requires_grad_(True)
    color, depth, trans = raster.rasterize(rast, poses, tau)
    P = intr.width * intr.height
    g = np.random.default_rng(4)
    wc, wd, wt = (g.normal(size=n) for n in (3 * P, P, P))
    tw = [torch.as_tensor(x.astype(np.float32), device="cuda") for x in (wc, wd, wt)]
    loss = (tw[0] * color).sum() + (tw[1] * depth).sum() + (tw[2] * trans).sum()
    loss.backward()
    got = tau.grad.reshape(-1).cpu().numpy()
    t64 = tau0.astype(np.float64)
    eff = left_perturb(pose.astype(np.float64), t64)
    wc32, wd32, wt32 = (x.astype(np.float32).astype(np.float64) for x in (wc, wd, wt))
    gpose = O.backward(sc, eff, intr, wc32.reshape(3, P), wd32, wt32)[3]
    ref = _numeric_left_jacobian(t64).T @ gpose

    def oracle_loss(t):
        c, d, tr = O.render(sc, left_perturb(pose.astype(np.float64), t), intr)
        return float((wc32.reshape(3, P) * c).sum() + (wd32 * d).sum() + (wt32 * tr).sum())

    h = 1e-6
    fd = np.array([(oracle_loss(t64 + h * np.eye(6)[k]) - oracle_loss(t64 - h * np.eye(6)[k])) / (2 * h)
                   for k in range(6)])
    ok_fd, msg_fd, _ = grad_close(ref, fd, rel=1e-4, abs_frac=1e-5, name="J_l^T g vs FD")
    _say("  " + msg_fd)
    assert ok_fd, msg_fd
    ok, msg, _ = grad_close(got, ref, name="tau.grad")
    _say("  " + msg)
    assert ok, msg


def test_autograd_backward_refuses_a_rebinned_workspace():
    """The Function keeps the binning in the rasterizer's workspace, so a second render on the
    same rasterizer before backward must make that backward fail loudly."""
    sc, intr = tiny_scene(23, n_faces=30)
    dev = raster.DeviceScene.from_numpy(sc)
    dev.pos.requires_grad_(True)
    rast = raster.Rasterizer(dev, [intr])
    poses = raster.poses_tensor([IDENTITY])
    rast.fit(poses)
    color, _, _ = raster.rasterize(rast, poses)
    other = raster.poses_tensor([left_perturb(IDENTITY, np.array([0.01, 0, 0, 0, 0.02, 0]))])
    raster.rasterize(rast, other)                     # re-bins the shared workspace
    with pytest.raises(RuntimeError, match="re-binned"):
        color.sum().backward()
    color2, _, _ = raster.rasterize(rast, poses)      # a fresh graph works
    color2.sum().backward()
    assert torch.isfinite(dev.pos.grad).all()


def test_soup_vertices_past_the_faces_get_zero_gradients():
    """A soup with more vertices than 3 M: the backward, the fused L1 step and the photometric
    step write zeros for the vertices past the faces' (outputs pre-filled with garbage)."""
    sc, intr = tiny_scene(24, n_faces=30)
    M = sc.n_faces
    g = np.random.default_rng(24)
    extra = 7
    pos = np.concatenate([sc.pos, g.uniform(-1, 1, (3, extra)).astype(np.float32)], axis=1)
    col = np.concatenate([sc.col, g.uniform(0, 1, (3, extra)).astype(np.float32)], axis=1)
    opa = np.concatenate([sc.opa, g.uniform(0.3, 1, extra).astype(np.float32)])
    dev = raster.DeviceScene.from_numpy(S.Scene(pos, col, opa, None))
    dev.n_faces = M                                   # faces 0..M-1; vertices 3M..3M+6 belong to none
    rast = raster.Rasterizer(dev, [intr])
    poses = raster.poses_tensor([IDENTITY])
    rast.fit(poses)
    N = 3 * M + extra
    P = intr.width * intr.height
    tc = torch.rand(3 * P, device="cuda")
    td = torch.rand(P, device="cuda") + 1.0

    def garbage():
        return [torch.full((3 * N,), 7.0, device="cuda"), torch.full((3 * N,), 7.0, device="cuda"),
                torch.full((N,), 7.0, device="cuda"), torch.full((6,), 7.0, device="cuda")]

    rast.bin_and_sort(poses)
    c, d, _ = rast.forward(poses)
    outs = {"backward": rast.backward(poses, torch.ones(3 * P, device="cuda"), torch.ones(P, device="cuda"),
                                      out=garbage()),
            "train_l1": rast.train_l1(poses, tc, td, out=garbage()),
            "photometric": rast.train_photometric(poses, tc, td, out=garbage())}
    torch.cuda.synchronize()
    for nm, (gp, gc, go, _) in outs.items():
        gp, gc = gp.view(3, N).cpu().numpy(), gc.view(3, N).cpu().numpy()
        go = go.cpu().numpy()
        assert np.all(gp[:, 3 * M:] == 0) and np.all(gc[:, 3 * M:] == 0) and np.all(go[3 * M:] == 0), nm
        assert np.all(np.isfinite(gp)) and not np.any(gp[:, :3 * M] == 7.0), nm


def test_autograd_keeps_no_per_pixel_lists():
    """The workspace grows by 8 bytes per pixel (last-face index, transmittance before it)
    plus per-tile bookkeeping (loss partials 16, counters 16, range 8, order 4 and long-list
    entry 4: 48 bytes) -- independent of how many faces cover a pixel."""
    sc, intr = tiny_scene(22, n_faces=40)
    dev = raster.DeviceScene.from_numpy(sc)
    small = raster.Rasterizer(dev, [S.Intrinsics(64, 64, 50.0, 50.0, 31.5, 31.5)])
    big = raster.Rasterizer(dev, [S.Intrinsics(128, 128, 50.0, 50.0, 63.5, 63.5)])
    d = big.workspace_bytes(0) - small.workspace_bytes(0)
    px = 128 * 128 - 64 * 64
    tiles = 64 - 16
    assert d <= 8 * px + 48 * tiles + 4 * 256, d


# ---------------------------------------------------------------------------- mapping window

def _room(n_faces, seed=31):
    return S.room_soup(seed, n_faces, size_range=(0.005, 0.03))


def _window_inputs(n_views=4, n_faces=60_000, w=320, h=240, seed=41):
    sc = _room(n_faces)
    g = S.rng(seed)
    poses = S.room_trajectory(g, n_views)
    intr = S.intrinsics_for(w, h)
    targets = [S.perturb_pose(p, g) for p in poses]
    dev = raster.DeviceScene.from_numpy(sc)
    tr = raster.Rasterizer(dev, [intr] * n_views)
    tp = raster.poses_tensor(targets)
    tr.fit(tp)
    tr.bin_and_sort(tp)
    tc, td, _ = tr.forward(tp)
    return sc, dev, poses, [intr] * n_views, tc.clone(), td.clone()


def test_window_batched_equals_sum_of_single_views():
    sc, dev, poses, intrs, tc, td = _window_inputs()
    win = MappingWindow(dev, intrs, schedule=(1, 1, 2048))
    p = raster.poses_tensor(poses)
    win.prepare(p)
    gp, gc, go, gpose = [x.clone() for x in win.step(p, tc, td, check_capacity=True)]
    loss_b = win.loss.clone()
    P = intrs[0].width * intrs[0].height
    acc = [torch.zeros_like(gp), torch.zeros_like(gc), torch.zeros_like(go)]
    for v in range(len(poses)):
        r = raster.Rasterizer(dev, [intrs[v]])
        pv = raster.poses_tensor([poses[v]])
        r.fit(pv)
        r.bin_and_sort(pv)
        lv = torch.zeros(1, device="cuda")
        a, b, c, d = r.train_l1(pv, tc[3 * P * v:3 * P * (v + 1)], td[P * v:P * (v + 1)], loss=lv)
        acc[0] += a; acc[1] += b; acc[2] += c
        np.testing.assert_allclose(d.cpu().numpy(), gpose[6 * v:6 * (v + 1)].cpu().numpy(), rtol=1e-3, atol=1e-9)
        np.testing.assert_allclose(lv.cpu().numpy(), loss_b[v:v + 1].cpu().numpy(), rtol=1e-5)
    for nm, a, b in zip(["pos", "col", "opa"], [gp, gc, go], acc):
        ok, msg, _ = grad_close(a.cpu().numpy(), b.cpu().numpy(), name=nm)
        _say("  " + msg)
        assert ok, msg


@pytest.mark.parametrize("w,h", [(320, 240), (1200, 680)], ids=["900_tiles", "9675_tiles"])
def test_every_schedule_gives_the_same_step(w, h):
    """Every schedule reproduces the one-workgroup-per-tile step.  The longest-first tile
    order is built with the binning for the 900-tile window and by its own kernel for the
    9675-tile one (above 8192 tiles)."""
    sc, dev, poses, intrs, tc, td = _window_inputs(n_views=3, n_faces=40_000, w=w, h=h)
    p = raster.poses_tensor(poses)
    win = MappingWindow(dev, intrs, schedule=(0, 0, 0))
    win.prepare(p)
    ref = [x.clone().cpu().numpy() for x in win.step(p, tc, td, check_capacity=True)]
    for cand in autotune.CANDIDATES[1:]:
        win.rast.schedule = cand
        got = [x.cpu().numpy() for x in win.step(p, tc, td)]
        for nm, a, b in zip(["pos", "col", "opa", "pose"], got, ref):
            ok, msg, _ = grad_close(a, b, rel=1e-4, name=f"{cand} {nm}")
            assert ok, msg


def test_autotuner_picks_and_records_a_schedule(tmp_path):
    sc, dev, poses, intrs, tc, td = _window_inputs(n_views=2, n_faces=30_000)
    p = raster.poses_tensor(poses)
    win = MappingWindow(dev, intrs, schedule=(0, 0, 0))
    k = win.prepare(p)
    best, times = autotune.tune(win.rast, p, tc, td, reps=3)
    assert best in autotune.CANDIDATES and len(times) == len(autotune.CANDIDATES)
    path = str(tmp_path / "table.json")
    tab = {}
    autotune.record(tab, intrs, k, best, times)
    autotune.save_table(tab, path)
    assert autotune.lookup(intrs, k, path) == best


# ---------------------------------------------------------------------------- tracking graph

def test_tracking_graph_replay_matches_eager():
    sc = _room(80_000, seed=33)
    g = S.rng(34)
    pose0 = S.random_room_pose(g)
    truth = S.perturb_pose(pose0, g)
    intr = S.intrinsics_for(320, 240)
    dev = raster.DeviceScene.from_numpy(sc)
    tr = raster.Rasterizer(dev, [intr])
    tp = raster.poses_tensor([truth])
    tr.fit(tp)
    tr.bin_and_sort(tp)
    tc, td, _ = tr.forward(tp)
    trk = Tracker(dev, intr, iters=30)
    p0 = torch.as_tensor(pose0, device="cuda")
    trk.set_frame(p0, tc, td)
    eager = trk.run_eager().clone()
    loss_eager = trk.loss_hist.clone()
    trk.check()
    trk.set_frame(p0, tc, td)
    trk.capture()
    trk.set_frame(p0, tc, td)
    for rep in range(3):                       # replay several times with eager work between
        trk.set_frame(p0, tc, td)
        out = trk.replay().clone()
        torch.cuda.synchronize()
        trk.check()
        _say(f"  replay {rep}: |pose - eager| = {np.abs(out.cpu().numpy() - eager.cpu().numpy()).max():.2e}")
        np.testing.assert_allclose(out.cpu().numpy(), eager.cpu().numpy(), atol=1e-5)
        np.testing.assert_allclose(trk.loss_hist.cpu().numpy(), loss_eager.cpu().numpy(), rtol=1e-4, atol=1e-8)
    lh = loss_eager.cpu().numpy()
    _say(f"  loss {lh[0]:.5f} -> {lh[-1]:.5f}")
    assert lh[-1] < lh[0]


def test_tracking_graph_with_dssim_matches_eager():
    """The full tracking energy (L1 colour 0.8, D-SSIM 0.2, depth 0.05) captured in a graph:
    replays equal the eager loop, and a small step along the pose gradient lowers the energy."""
    sc = _room(60_000, seed=39)
    g = S.rng(40)
    pose0 = S.random_room_pose(g)
    truth = S.perturb_pose(pose0, g)
    intr = S.intrinsics_for(320, 240)
    dev = raster.DeviceScene.from_numpy(sc)
    tr = raster.Rasterizer(dev, [intr])
    tp = raster.poses_tensor([truth])
    tr.fit(tp)
    tr.bin_and_sort(tp)
    tc, td, _ = tr.forward(tp)
    trk = Tracker(dev, intr, iters=20, w_ssim=0.2)
    p0 = torch.as_tensor(pose0, device="cuda")
    trk.set_frame(p0, tc, td)
    eager = trk.run_eager().clone()
    loss_eager = trk.loss_hist.clone()
    trk.set_frame(p0, tc, td)
    trk.capture()
    for rep in range(2):
        trk.set_frame(p0, tc, td)
        out = trk.replay().clone()
        torch.cuda.synchronize()
        trk.check()
        np.testing.assert_allclose(out.cpu().numpy(), eager.cpu().numpy(), atol=1e-5)
        np.testing.assert_allclose(trk.loss_hist.cpu().numpy(), loss_eager.cpu().numpy(), rtol=1e-4, atol=1e-8)
    lh = loss_eager.cpu().numpy()
    _say(f"  loss {lh[0]:.5f} -> {lh[-1]:.5f} (plain gradient steps at the L1 learning rates)")
    # first-order descent: a small step along the negative gradient lowers the full energy
    small = Tracker(dev, intr, iters=2, w_ssim=0.2, lr_trans=1e-5, lr_rot=3e-5)
    small.set_frame(p0, tc, td)
    small.run_eager()
    sh = small.loss_hist.cpu().numpy()
    _say(f"  small step: {sh[0]:.7f} -> {sh[1]:.7f}")
    assert sh[1] < sh[0]


@pytest.mark.parametrize("w,h", [(320, 240), (1200, 680)], ids=["900_tiles", "9675_tiles"])
def test_window_with_dssim_equals_sum_of_single_views(w, h):
    """The separate forward and backward of the D-SSIM step walk the tiles longest-first: with
    the order built by the binning (900 tiles, and each single view) or, above 8192 tiles, by
    its own kernel (9675 tiles)."""
    sc, dev, poses, intrs, tc, td = _window_inputs(n_views=3, n_faces=40_000, w=w, h=h)
    win = MappingWindow(dev, intrs, w_ssim=0.2)
    p = raster.poses_tensor(poses)
    win.prepare(p)
    gp, gc, go, gpose = [x.clone() for x in win.step(p, tc, td, check_capacity=True)]
    loss_b = win.loss.clone()
    P = intrs[0].width * intrs[0].height
    acc = [torch.zeros_like(gp), torch.zeros_like(gc), torch.zeros_like(go)]
    for v in range(len(poses)):
        r = raster.Rasterizer(dev, [intrs[v]])
        pv = raster.poses_tensor([poses[v]])
        r.fit(pv)
        r.bin_and_sort(pv)
        lv = torch.zeros(1, device="cuda")
        a, b, c, d = r.train_photometric(pv, tc[3 * P * v:3 * P * (v + 1)], td[P * v:P * (v + 1)], loss=lv)
        acc[0] += a; acc[1] += b; acc[2] += c
        np.testing.assert_allclose(d.cpu().numpy(), gpose[6 * v:6 * (v + 1)].cpu().numpy(), rtol=1e-3, atol=1e-9)
        np.testing.assert_allclose(lv.cpu().numpy(), loss_b[v:v + 1].cpu().numpy(), rtol=1e-5)
    for nm, a, b in zip(["pos", "col", "opa"], [gp, gc, go], acc):
        ok, msg, _ = grad_close(a.cpu().numpy(), b.cpu().numpy(), name=nm)
        _say("  " + msg)
        assert ok, msg


def test_window_mapping_energy_is_the_sum_of_its_terms():
    """The window step with D-SSIM, E_equi and E_norm (weights 0.2, 1.2, 0.05; target normals
    from the target depth) equals the photometric step plus the separately computed
    equilateral and normal-loss gradients."""
    sc, dev, poses, intrs, tc, td = _window_inputs(n_views=3, n_faces=30_000)
    p = raster.poses_tensor(poses)
    tn = raster.sensor_normals(td, intrs)
    win = MappingWindow(dev, intrs, w_ssim=0.2, w_equi=1.2, w_norm=0.05)
    win.prepare(p)
    got = [x.clone() for x in win.step(p, tc, td, check_capacity=True, target_normals=tn)]
    torch.cuda.synchronize()
    base = MappingWindow(dev, intrs, w_ssim=0.2)
    base.prepare(p)
    b = [x.clone() for x in base.step(p, tc, td, check_capacity=True)]
    le, ge = raster.equilateral(dev, weight=1.2)
    nr = raster.Rasterizer(dev, intrs)
    nr.fit(p)
    ln = torch.zeros(len(intrs), device="cuda")
    gnp, gno, gnpose = nr.train_normal(p, tn, w_norm=0.05, loss=ln)
    torch.cuda.synchronize()
    want = [b[0] + ge.reshape(-1) + gnp, b[1], b[2] + gno, b[3] + gnpose]
    for nm, a, w in zip(["pos", "col", "opa", "pose"], got, want):
        ok, msg, _ = grad_close(a.cpu().numpy(), w.cpu().numpy(), name=nm)
        _say("  " + msg)
        assert ok, msg
    np.testing.assert_allclose(win.equi_loss.cpu().numpy(), le.cpu().numpy(), rtol=1e-6)
    np.testing.assert_allclose(win.norm_loss.cpu().numpy(), ln.cpu().numpy(), rtol=1e-5)
    _say(f"  E_equi {float(le):.5f}, E_norm per view {ln.cpu().numpy()}")


# ---------------------------------------------------------------------------- serving

def test_served_results_equal_alone_results():
    sc = _room(100_000, seed=35)
    dev = raster.DeviceScene.from_numpy(sc)
    queries = S.serving_queries(36, 24, qps=1e6)
    ex = GpuExecutor(dev, pairs_per_tile=20.0)        # small estimate: exercises the overflow retry
    srv = Server(ex, n_slots=3, mem_budget=3 << 30, max_batch_views=6)
    srv.start()
    try:
        reqs = [srv.submit(Request(i, intr, pose)) for i, (_, intr, pose) in enumerate(queries)]
        srv.drain()
    finally:
        srv.stop()
    assert all(r.error is None for r in reqs), [r.error for r in reqs if r.error]
    _say(f"  stats {srv.stats()} retries {ex.retries}")
    for r in reqs:
        c, d, _ = G.render(*G.make(sc, [r.intr], [r.pose]))
        W, H = r.intr.width, r.intr.height
        assert np.array_equal(r.color.cpu().numpy().reshape(-1), c.reshape(-1)), r.rid
        assert np.array_equal(r.depth.cpu().numpy().reshape(-1), d.reshape(-1)), r.rid


def test_serving_under_a_tight_memory_budget():
    """Two one-view slots and room for one more 1200 x 680 output: the slot workspaces plus the
    admitted outputs stay within the budget -- in the server's books and in the device memory
    torch allocates while serving (outputs dropped at completion) -- and every query is served."""
    sc = _room(200_000, seed=37)
    dev = raster.DeviceScene.from_numpy(sc)
    queries = S.serving_queries(38, 40, qps=1e6)
    ex = GpuExecutor(dev)
    intr = S.intrinsics_for(1200, 680)
    out1 = ex.OUT_BYTES_PER_PIXEL * intr.width * intr.height
    ws1 = ex.slot_workspace_bytes(1)
    budget = 2 * (ws1 + out1) + out1
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    srv = Server(ex, n_slots=2, mem_budget=budget, max_batch_views=4, keep_outputs=False)
    srv.start()
    try:
        assert srv.max_views == 1 and srv.fixed == 2 * ws1
        reqs = [srv.submit(Request(i, intr_q, pose)) for i, (_, intr_q, pose) in enumerate(queries)]
        srv.drain()
    finally:
        srv.stop()
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() - base
    st = srv.stats()
    _say(f"  budget {budget / 2**20:.1f} MiB, books peak {srv.peak_used / 2**20:.1f} MiB, "
         f"allocated peak {peak / 2**20:.1f} MiB, {st}")
    assert all(r.error is None for r in reqs), [r.error for r in reqs if r.error]
    assert srv.peak_used <= budget and srv.used == 0
    assert peak <= budget


def test_mapping_window_takes_the_tabulated_schedule():
    """A window built without a schedule looks its workload up in the packaged table (written
    on this GPU model by tune_table.py) and runs that schedule."""
    w = S.workload("window_8x1200x680")
    dev = raster.DeviceScene.from_numpy(w.scene)
    win = MappingWindow(dev, w.intr)
    k = win.prepare(raster.poses_tensor(w.poses))
    want = autotune.lookup(w.intr, k)
    _say(f"  K = {k}, key {autotune.key_for(w.intr, k)}, schedule {win.schedule}")
    assert want is not None and win.schedule == want and win.rast.schedule == want
