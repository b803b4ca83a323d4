"""PyTorch-facing API of the rasterizer.  PyTorch supplies device memory and streams only;
every computation runs in the HIP kernels behind the C ABI (``_lib``).

Main entry points
  * ``Rasterizer``: holds parameters and a workspace; ``bin_and_sort`` / ``forward`` /
    ``backward`` / ``train_l1`` map one-to-one onto the C ABI calls.
  * ``rasterize``: differentiable render through ``TriangleRasterFn`` (autograd), with an
    optional se(3) left perturbation ``tau`` per view whose gradient is the pose gradient.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib
from ._lib import TsrBinning, TsrIntrinsics, TsrParams, TsrScene, TsrSchedule, check


@dataclasses.dataclass
class Params:
    """Rendering parameters (window exponent of eq. 3, early-stop threshold, culling, the L1
    weights of the fused training loss: 0.8 = 1 - lambda of eq. 8, 0.05 = lambda_dep, and the
    face-opacity rule)."""
    sigma: float = 1.0
    t_min: float = 1e-6
    z_near: float = 0.1
    r_min: float = 1e-3
    w_color: float = 0.8
    w_depth: float = 0.05
    opacity_min: bool = False     # face opacity = min of the vertex opacities (Mesh Splatting variant)
    tight_tiles: bool = False     # list a face only in the tiles that can hold a pixel it covers
    perspective: bool = False     # perspective-correct colour interpolation and plane depth

    def c(self) -> TsrParams:
        return TsrParams(self.sigma, self.t_min, self.z_near, self.r_min, self.w_color, self.w_depth,
                         1 if self.opacity_min else 0, 1 if self.tight_tiles else 0, 1 if self.perspective else 0)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def intrinsics_array(intrs: Sequence) -> C.Array:
    arr = (TsrIntrinsics * len(intrs))()
    for i, it in enumerate(intrs):
        w, h, fx, fy, cx, cy = it.as_tuple() if hasattr(it, "as_tuple") else it
        arr[i] = TsrIntrinsics(int(w), int(h), fx, fy, cx, cy)
    return arr


class DeviceScene:
    """Scene arrays resident on the device (SoA float32, optional int32 faces)."""

    def __init__(self, pos: torch.Tensor, col: torch.Tensor, opa: torch.Tensor,
                 faces: Optional[torch.Tensor] = None, face_sigma: Optional[torch.Tensor] = None):
        for name, t in (("pos", pos), ("col", col), ("opa", opa)) + ((("face_sigma", face_sigma),)
                                                                     if face_sigma is not None else ()):
            if t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        self.pos, self.col, self.opa = pos, col, opa
        self.faces = faces
        self.n_vertices = int(pos.shape[1])
        self.n_faces = int(faces.shape[0]) if faces is not None else self.n_vertices // 3
        # per-face window exponents (Triangle Splatting variant), or None for the global sigma
        self.face_sigma = face_sigma
        if face_sigma is not None and face_sigma.numel() != self.n_faces:
            raise ValueError(f"face_sigma needs {self.n_faces} values")

    @classmethod
    def from_numpy(cls, scene, device="cuda") -> "DeviceScene":
        f = None if scene.faces is None else torch.as_tensor(scene.faces, dtype=torch.int32, device=device).contiguous()
        fs = getattr(scene, "face_sigma", None)
        fs = None if fs is None else torch.as_tensor(np.asarray(fs, np.float32), device=device).contiguous()
        return cls(torch.as_tensor(scene.pos, device=device).contiguous(),
                   torch.as_tensor(scene.col, device=device).contiguous(),
                   torch.as_tensor(scene.opa, device=device).contiguous(), f, fs)

    def c(self) -> TsrScene:
        return TsrScene(self.pos.data_ptr(), self.col.data_ptr(), self.opa.data_ptr(),
                        None if self.faces is None else self.faces.data_ptr(), self.n_vertices, self.n_faces,
                        None if self.face_sigma is None else self.face_sigma.data_ptr(), None)


def poses_tensor(poses, device="cuda") -> torch.Tensor:
    if isinstance(poses, torch.Tensor):
        return poses.to(device=device, dtype=torch.float32).reshape(-1, 12).contiguous()
    return torch.as_tensor(np.stack([np.asarray(p, np.float32).reshape(12) for p in poses]),
                           device=device).contiguous()


class Rasterizer:
    """One workspace plus the C ABI calls on it.  The workspace is grown on demand when the
    binning reports a capacity overflow (one synchronising check per bin when
    ``check_capacity`` is set)."""

    def __init__(self, scene: DeviceScene, intrs: Sequence, params: Optional[Params] = None,
                 capacity: int = 0, device="cuda", workspace: Optional[torch.Tensor] = None):
        self.lib = _lib.load()
        self.scene = scene
        self.intrs = list(intrs)
        self.n_views = len(self.intrs)
        self.params = params or Params()
        self._cintr = intrinsics_array(self.intrs)
        self._cscene = scene.c()
        self._cparams = self.params.c()
        self.device = device
        self.pixels = [int(i.width) * int(i.height) for i in self.intrs]
        self.total_pixels = sum(self.pixels)
        self.ws: Optional[torch.Tensor] = None
        self.capacity = 0
        self.schedule: Optional[Tuple[int, int, int]] = None   # (persistent, order, grid) for train_l1
        # bumped by every call that rewrites the binning or the per-pixel state in the workspace
        # (the autograd Function checks it between its forward and backward)
        self.generation = 0
        # dL/dsigma_m of the latest backward when the scene has per-face exponents
        self.grad_face_sigma = (torch.empty(scene.n_faces, device=device) if scene.face_sigma is not None
                                else None)
        if workspace is not None and workspace.numel() >= self.workspace_bytes(capacity):
            # caller-provided buffer (e.g. reused across requests): use all of it
            self.ws = workspace
            self.capacity = self._capacity_of(workspace.numel())
            check(self.lib.tsr_workspace_init(_ptr(self.ws), C.c_size_t(self.ws.numel()), _stream()),
                  "tsr_workspace_init")
        else:
            self.ensure_capacity(capacity)

    def _capacity_of(self, nbytes: int) -> int:
        """Largest pair capacity a buffer of nbytes holds (16 bytes per pair beyond the fixed part)."""
        fixed = self.workspace_bytes(0)
        cap = max(0, (nbytes - fixed) // 16)
        while cap > 0 and self.workspace_bytes(cap) > nbytes:
            cap -= 1
        return int(cap)

    # ----------------------------------------------------------------- workspace
    def workspace_bytes(self, capacity: int) -> int:
        out = C.c_size_t(0)
        check(self.lib.tsr_workspace_size(C.byref(self._cscene), self._cintr, self.n_views, int(capacity),
                                          C.byref(out)), "tsr_workspace_size")
        return int(out.value)

    def ensure_capacity(self, capacity: int) -> None:
        if self.ws is not None and capacity <= self.capacity:
            return
        nbytes = self.workspace_bytes(capacity)
        self.generation += 1
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.capacity = int(capacity)
        check(self.lib.tsr_workspace_init(_ptr(self.ws), C.c_size_t(nbytes), _stream()), "tsr_workspace_init")

    def _args(self, poses: torch.Tensor):
        return (C.byref(self._cscene), _ptr(poses), self._cintr, self.n_views, C.byref(self._cparams),
                _ptr(self.ws), C.c_size_t(self.ws.numel()))

    def count(self, poses: torch.Tensor, stream=None) -> int:
        self.generation += 1
        k = C.c_int64(0)
        check(self.lib.tsr_count(*self._args(poses), _stream(stream), C.byref(k)), "tsr_count")
        return int(k.value)

    def fit(self, poses: torch.Tensor, slack: float = 1.25) -> int:
        """Size the workspace for these poses from an exact pair count."""
        k = self.count(poses)
        self.ensure_capacity(int(k * slack) + 4096)
        return k

    # ----------------------------------------------------------------- C ABI calls
    def bin_and_sort(self, poses: torch.Tensor, stream=None, check_capacity: bool = True) -> None:
        self.generation += 1
        check(self.lib.tsr_bin_and_sort(*self._args(poses), _stream(stream)), "tsr_bin_and_sort")
        if check_capacity:
            rc = self.lib.tsr_check(_ptr(self.ws), _stream(stream), None)
            if rc == _lib.TSR_ECAPACITY:
                self.fit(poses)
                check(self.lib.tsr_bin_and_sort(*self._args(poses), _stream(stream)), "tsr_bin_and_sort")
                check(self.lib.tsr_check(_ptr(self.ws), _stream(stream), None), "tsr_check")
            else:
                check(rc, "tsr_check")

    def forward(self, poses: torch.Tensor, color=None, depth=None, trans=None, stream=None):
        self.generation += 1
        P = self.total_pixels
        color = color if color is not None else torch.empty(3 * P, device=self.device)
        depth = depth if depth is not None else torch.empty(P, device=self.device)
        trans = trans if trans is not None else torch.empty(P, device=self.device)
        check(self.lib.tsr_render_forward(*self._args(poses), _ptr(color), _ptr(depth), _ptr(trans), _stream(stream)),
              "tsr_render_forward")
        return color, depth, trans

    def grad_buffers(self, want=(True, True, True, True)):
        N = self.scene.n_vertices
        gp = torch.empty(3 * N, device=self.device) if want[0] else None
        gc = torch.empty(3 * N, device=self.device) if want[1] else None
        go = torch.empty(N, device=self.device) if want[2] else None
        gpose = torch.empty(6 * self.n_views, device=self.device) if want[3] else None
        return gp, gc, go, gpose

    def _sigma_out(self, grad_face_sigma: Optional[torch.Tensor]) -> None:
        """Points the scene's dL/dsigma output at `grad_face_sigma` (default: this rasterizer's
        buffer) when the scene has per-face exponents."""
        if self.scene.face_sigma is not None:
            buf = grad_face_sigma if grad_face_sigma is not None else self.grad_face_sigma
            self._cscene.grad_face_sigma = buf.data_ptr()

    def backward(self, poses: torch.Tensor, grad_color, grad_depth, grad_trans=None, out=None, stream=None,
                 grad_face_sigma=None):
        gp, gc, go, gpose = out if out is not None else self.grad_buffers()
        self._sigma_out(grad_face_sigma)
        check(self.lib.tsr_render_backward(*self._args(poses), _ptr(grad_color), _ptr(grad_depth), _ptr(grad_trans),
                                           _ptr(gp), _ptr(gc), _ptr(go), _ptr(gpose), _stream(stream)),
              "tsr_render_backward")
        return gp, gc, go, gpose

    def train_l1(self, poses: torch.Tensor, target_color, target_depth, color=None, depth=None, trans=None,
                 loss=None, out=None, schedule=None, stream=None):
        self.generation += 1
        gp, gc, go, gpose = out if out is not None else self.grad_buffers()
        self._sigma_out(None)
        sched = self.schedule if schedule is None else schedule
        sp = None if sched is None else C.byref(TsrSchedule(*sched))
        check(self.lib.tsr_render_train_l1(*self._args(poses), _ptr(target_color), _ptr(target_depth), _ptr(color),
                                           _ptr(depth), _ptr(trans), _ptr(loss), _ptr(gp), _ptr(gc), _ptr(go),
                                           _ptr(gpose), sp, _stream(stream)), "tsr_render_train_l1")
        return gp, gc, go, gpose

    def photometric_scratch(self) -> torch.Tensor:
        """Scratch of the D-SSIM statistics and per-pixel seeds (allocated on first use)."""
        if getattr(self, "_pscratch", None) is None:
            nb = C.c_size_t()
            check(self.lib.tsr_dssim_scratch_size(self._cintr, self.n_views, C.byref(nb)), "tsr_dssim_scratch_size")
            self._pscratch = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        return self._pscratch

    def train_photometric(self, poses: torch.Tensor, target_color, target_depth, w_ssim: float = 0.2,
                          color=None, depth=None, trans=None, loss=None, out=None, stream=None):
        """Forward, the full loss of eqs. 8 and 10 (L1 colour, D-SSIM, masked L1 depth) and its
        backward (``tsr_render_train_photometric``)."""
        self.generation += 1
        P = self.total_pixels
        color = color if color is not None else torch.empty(3 * P, device=self.device)
        depth = depth if depth is not None else torch.empty(P, device=self.device)
        gp, gc, go, gpose = out if out is not None else self.grad_buffers()
        self._sigma_out(None)
        sc = self.photometric_scratch()
        check(self.lib.tsr_render_train_photometric(*self._args(poses), _ptr(target_color), _ptr(target_depth),
                                                    float(w_ssim), _ptr(color), _ptr(depth), _ptr(trans), _ptr(loss),
                                                    _ptr(gp), _ptr(gc), _ptr(go), _ptr(gpose), _ptr(sc),
                                                    C.c_size_t(sc.numel()), _stream(stream)),
              "tsr_render_train_photometric")
        return gp, gc, go, gpose

    def face_stats(self, poses: torch.Tensor, want=(True, True, True), stream=None):
        """Per-(view, face) projected area, dominant-pixel coverage and visibility
        (``tsr_face_stats``), each [V * M] or None; coverage and visibility use the binning held
        in the workspace (call ``bin_and_sort`` with the same poses first)."""
        n = self.n_views * self.scene.n_faces
        area = torch.empty(n, device=self.device) if want[0] else None
        cov = torch.empty(n, dtype=torch.int32, device=self.device) if want[1] else None
        vis = torch.empty(n, dtype=torch.int32, device=self.device) if want[2] else None
        check(self.lib.tsr_face_stats(*self._args(poses), _ptr(area), _ptr(cov), _ptr(vis), _stream(stream)),
              "tsr_face_stats")
        return area, cov, vis

    def train_normal(self, poses: torch.Tensor, target_normals: torch.Tensor, w_norm: float = 0.05,
                     normal_map=None, loss=None, out=None, accumulate: bool = False, stream=None):
        """Normal loss of mapping (``tsr_render_train_normal``): bins, renders the normal map
        and back-propagates w_norm * mean(1 - N . N_bar); returns (grad_pos, grad_opa,
        grad_pose), written or (``accumulate``) added into ``out``.  Leaves the workspace binned
        for the normal-coloured soup."""
        self.generation += 1
        if getattr(self, "_nscratch", None) is None:
            nb = C.c_size_t()
            check(self.lib.tsr_normal_scratch_size(C.byref(self._cscene), self._cintr, self.n_views, C.byref(nb)),
                  "tsr_normal_scratch_size")
            self._nscratch = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        if out is None:
            if accumulate:
                raise ValueError("accumulate needs the gradient buffers")
            gp, _, go, gpose = self.grad_buffers((True, False, True, True))
        else:
            gp, go, gpose = out
        sc = self._nscratch
        check(self.lib.tsr_render_train_normal(*self._args(poses), _ptr(target_normals), float(w_norm),
                                               _ptr(normal_map), _ptr(loss), _ptr(gp), _ptr(go), _ptr(gpose),
                                               1 if accumulate else 0, _ptr(sc), C.c_size_t(sc.numel()),
                                               _stream(stream)),
              "tsr_render_train_normal")
        return gp, go, gpose

    def mapping_scratch(self) -> torch.Tensor:
        """Scratch of the one-binning mapping step (allocated on first use)."""
        if getattr(self, "_mscratch", None) is None:
            nb = C.c_size_t()
            check(self.lib.tsr_mapping_scratch_size(C.byref(self._cscene), self._cintr, self.n_views, C.byref(nb)),
                  "tsr_mapping_scratch_size")
            self._mscratch = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        return self._mscratch

    def train_mapping(self, poses: torch.Tensor, target_color, target_depth, target_normals, w_ssim: float = 0.2,
                      w_norm: float = 0.05, color=None, depth=None, trans=None, normal_map=None, loss=None,
                      loss_norm=None, out=None, grad_face_sigma=None, stream=None):
        """The photometric, depth and normal terms of the mapping energy on the binning held in
        the workspace (``tsr_render_train_mapping``: one forward that also composites the normal
        map, one backward that takes all seeds).  Returns (grad_pos, grad_col, grad_opa,
        grad_pose) of the sum of both per-view losses, overwriting ``out``."""
        self.generation += 1
        P = self.total_pixels
        color = color if color is not None else torch.empty(3 * P, device=self.device)
        depth = depth if depth is not None else torch.empty(P, device=self.device)
        gp, gc, go, gpose = out if out is not None else self.grad_buffers()
        self._sigma_out(grad_face_sigma)
        sc = self.mapping_scratch()
        check(self.lib.tsr_render_train_mapping(*self._args(poses), _ptr(target_color), _ptr(target_depth),
                                                _ptr(target_normals), float(w_ssim), float(w_norm), _ptr(color),
                                                _ptr(depth), _ptr(trans), _ptr(normal_map), _ptr(loss),
                                                _ptr(loss_norm), _ptr(gp), _ptr(gc), _ptr(go), _ptr(gpose), _ptr(sc),
                                                C.c_size_t(sc.numel()), _stream(stream)),
              "tsr_render_train_mapping")
        return gp, gc, go, gpose

    def pose_step(self, poses: torch.Tensor, grad_pose: torch.Tensor, lr_trans: float, lr_rot: float,
                  stream=None) -> None:
        check(self.lib.tsr_pose_step(_ptr(poses), _ptr(grad_pose), self.n_views, lr_trans, lr_rot, _stream(stream)),
              "tsr_pose_step")

    def binning(self) -> TsrBinning:
        b = TsrBinning()
        check(self.lib.tsr_binning_view(C.byref(self._cscene), self._cintr, self.n_views, _ptr(self.ws),
                                        C.c_size_t(self.ws.numel()), C.byref(b)), "tsr_binning_view")
        return b

    # ----------------------------------------------------------------- helpers
    def split_views(self, flat: torch.Tensor, channels: int) -> List[torch.Tensor]:
        """Unpack a packed per-view output into [channels, H, W] views."""
        out, off = [], 0
        for it in self.intrs:
            n = int(it.width) * int(it.height) * channels
            out.append(flat[off:off + n].view(channels, int(it.height), int(it.width)))
            off += n
        return out

    def pack(self, per_view: Sequence[torch.Tensor]) -> torch.Tensor:
        return torch.cat([t.reshape(-1) for t in per_view]).contiguous()


class DSsim:
    """D-SSIM term of eq. (8) on packed colour images (``tsr_dssim``): per-view loss
    1 - mean SSIM and ``weight`` times its colour gradient, written or added into ``grad``."""

    def __init__(self, intrs: Sequence, device: str = "cuda"):
        self.lib = _lib.load()
        self.intrs = list(intrs)
        self.n_views = len(self.intrs)
        self.device = device
        self._cintr = intrinsics_array(self.intrs)
        self.n_values = 3 * sum(int(it.width) * int(it.height) for it in self.intrs)
        nb = C.c_size_t()
        check(self.lib.tsr_dssim_scratch_size(self._cintr, self.n_views, C.byref(nb)), "tsr_dssim_scratch_size")
        self.scratch = torch.empty(nb.value, dtype=torch.uint8, device=device)

    def _want(self, name: str, t: torch.Tensor, n: int) -> None:
        if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != n or t.device.type != "cuda":
            raise ValueError(f"{name}: need a contiguous float32 device tensor of {n} values")

    def __call__(self, color: torch.Tensor, target: torch.Tensor, weight: float = 1.0, loss=None, grad=None,
                 want_grad: bool = True, accumulate: bool = False, stream=None):
        self._want("color", color, self.n_values)
        self._want("target", target, self.n_values)
        loss = loss if loss is not None else torch.empty(self.n_views, device=self.device)
        if want_grad and grad is None:
            if accumulate:
                raise ValueError("accumulate needs a grad buffer")
            grad = torch.empty(self.n_values, device=self.device)
        if grad is not None:
            self._want("grad", grad, self.n_values)
        check(self.lib.tsr_dssim(self._cintr, self.n_views, _ptr(color), _ptr(target), float(weight),
                                 1 if accumulate else 0, _ptr(loss), _ptr(grad), _ptr(self.scratch),
                                 C.c_size_t(self.scratch.numel()), _stream(stream)), "tsr_dssim")
        return loss, grad


def equilateral(scene: DeviceScene, weight: float = 1.0, grad: Optional[torch.Tensor] = None,
                accumulate: bool = False, want_grad: bool = True, loss: Optional[torch.Tensor] = None,
                stream=None, noalloc: bool = False):
    """Equilateral regulariser of eq. (14) (``tsr_equilateral``): returns (loss [1], grad [3, N]
    or None), the gradient scaled by ``weight`` and written or added into ``grad``.  With
    ``noalloc`` the call goes to ``tsr_equilateral_noalloc`` (no scratch buffer; the library's
    static per-device partials, up to TSR_EQUI_NOALLOC_MAX_FACES faces)."""
    lib = _lib.load()
    dev = scene.pos.device
    scratch = None
    if not noalloc:
        nb = C.c_size_t()
        check(lib.tsr_equilateral_scratch_size(scene.n_faces, C.byref(nb)), "tsr_equilateral_scratch_size")
        scratch = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    loss = loss if loss is not None else torch.empty(1, device=dev)
    if want_grad and grad is None:
        if accumulate:
            raise ValueError("accumulate needs a grad buffer")
        grad = torch.empty(3, scene.n_vertices, device=dev)
    if grad is not None and (grad.dtype != torch.float32 or not grad.is_contiguous()
                             or grad.numel() != 3 * scene.n_vertices):
        raise ValueError("grad: need a contiguous float32 tensor of 3 * n_vertices values")
    sc = scene.c()
    if noalloc:
        check(lib.tsr_equilateral_noalloc(C.byref(sc), float(weight), 1 if accumulate else 0, _ptr(loss), _ptr(grad),
                                          _stream(stream)), "tsr_equilateral_noalloc")
    else:
        check(lib.tsr_equilateral(C.byref(sc), float(weight), 1 if accumulate else 0, _ptr(loss), _ptr(grad),
                                  _ptr(scratch), C.c_size_t(scratch.numel()), _stream(stream)), "tsr_equilateral")
    return loss, grad


def sensor_normals(depth: torch.Tensor, intrs: Sequence, normals: Optional[torch.Tensor] = None, stream=None):
    """Sensor normals of packed depth maps (``tsr_sensor_normals``), packed like colour; a
    zero vector marks an invalid pixel."""
    lib = _lib.load()
    n = sum(int(it.width) * int(it.height) for it in intrs)
    if depth.dtype != torch.float32 or not depth.is_contiguous() or depth.numel() != n:
        raise ValueError(f"depth: need a contiguous float32 tensor of {n} values")
    normals = normals if normals is not None else torch.empty(3 * n, device=depth.device)
    check(lib.tsr_sensor_normals(_ptr(depth), intrinsics_array(intrs), len(intrs), _ptr(normals), _stream(stream)),
          "tsr_sensor_normals")
    return normals


# ---------------------------------------------------------------------------- autograd

def compose_poses(tau: torch.Tensor, poses: torch.Tensor, stream=None) -> torch.Tensor:
    """Poses of Exp(tau) o T for tau [V, 6] = (rho, theta) (``tsr_pose_compose``)."""
    lib = _lib.load()
    tau = tau.detach().to(torch.float32).contiguous()
    poses = poses.detach().to(torch.float32).reshape(-1, 12).contiguous()
    if tau.shape != (poses.shape[0], 6):
        raise ValueError(f"tau must be [{poses.shape[0]}, 6]")
    out = torch.empty_like(poses)
    check(lib.tsr_pose_compose(_ptr(tau), _ptr(poses), poses.shape[0], _ptr(out), _stream(stream)),
          "tsr_pose_compose")
    return out


def tau_gradient(tau: torch.Tensor, grad_pose: torch.Tensor, stream=None) -> torch.Tensor:
    """dL/dtau = J_l(tau)^T grad_pose for a loss evaluated at Exp(tau) o T (``tsr_pose_tau_grad``)."""
    lib = _lib.load()
    tau = tau.detach().to(torch.float32).contiguous()
    g = grad_pose.detach().to(torch.float32).reshape(-1, 6).contiguous()
    out = torch.empty_like(g)
    check(lib.tsr_pose_tau_grad(_ptr(tau), _ptr(g), g.shape[0], _ptr(out), _stream(stream)), "tsr_pose_tau_grad")
    return out


class TriangleRasterFn(torch.autograd.Function):
    """Differentiable render: forward = bin_and_sort + render_forward (the workspace keeps
    the binning and each pixel's last-face state, not per-pixel blend lists); backward =
    render_backward (transmittance recovered by division, Sec. 3.3).  The pose enters as
    Exp(tau) o T (eq. 6); the pose gradient of the composed pose is mapped to tau through the
    left Jacobian of SE(3), so tau need not be zero.  The backward refuses to run once the
    rasterizer's workspace has been re-binned or re-rendered by another call."""

    @staticmethod
    def forward(ctx, pos, col, opa, face_sigma, tau, rast: Rasterizer, poses: torch.Tensor):
        eff = poses if tau is None else compose_poses(tau, poses)
        rast.bin_and_sort(eff)
        color, depth, trans = rast.forward(eff)
        ctx.rast = rast
        ctx.generation = rast.generation
        ctx.save_for_backward(eff, tau.detach() if tau is not None else None)
        ctx.has_tau = tau is not None
        return color, depth, trans

    @staticmethod
    def backward(ctx, g_color, g_depth, g_trans):
        eff, tau = ctx.saved_tensors
        rast: Rasterizer = ctx.rast
        if rast.generation != ctx.generation:
            raise RuntimeError("TriangleRasterFn.backward: the rasterizer's workspace was re-binned or re-rendered "
                               "after this forward (call backward before the next render, or use one Rasterizer "
                               "per pending graph)")
        g_color = g_color.contiguous() if g_color is not None else torch.zeros(3 * rast.total_pixels, device=eff.device)
        g_depth = g_depth.contiguous() if g_depth is not None else torch.zeros(rast.total_pixels, device=eff.device)
        g_trans = g_trans.contiguous() if g_trans is not None else None
        gsig = torch.empty_like(rast.scene.face_sigma) if rast.scene.face_sigma is not None else None
        gp, gc, go, gpose = rast.backward(eff, g_color, g_depth, g_trans, grad_face_sigma=gsig)
        N = rast.scene.n_vertices
        gtau = tau_gradient(tau, gpose) if ctx.has_tau else None
        return gp.view(3, N), gc.view(3, N), go.view(N), gsig, gtau, None, None


def rasterize(rast: Rasterizer, poses: torch.Tensor, tau: Optional[torch.Tensor] = None):
    """Differentiable colour [3P], depth [P], transmittance [P] (packed per view) of the
    rasterizer's scene.  Gradients flow to rast.scene.pos / col / opa (when they require
    grad), to rast.scene.face_sigma (per-face window exponents, when the scene has them) and
    to ``tau`` ([V, 6] se(3) left perturbation: the scene is rendered at Exp(tau) o T_CW)."""
    sc = rast.scene
    return TriangleRasterFn.apply(sc.pos, sc.col, sc.opa, sc.face_sigma, tau, rast, poses)
