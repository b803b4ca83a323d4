"""Tracking: camera-pose gradient descent against a fixed map (Sec. 3.4, tracking).

Each iteration is [bin and sort -> fused forward + L1 loss + backward (pose gradient only)
-> device-side pose step T <- Exp(-(lr_t g_rho, lr_r g_theta)) T], with the paper's learning
rates (translation 0.001, rotation 0.003) and 100 iterations per frame.  The whole loop can be
captured once into a HIP graph (through torch.cuda.graph) and replayed: no host
synchronisation happens inside it, every buffer is pre-sized, and the binning capacity is
checked after the replay through the device-side overflow flag.

With ``w_ssim > 0`` the loss is the full tracking energy of eqs. 8 and 10 (w_color L1 colour +
w_ssim D-SSIM + w_depth masked L1 depth; the paper uses 0.8, 0.2 and 0.05): forward, seeds and
backward then run as separate passes (``tsr_render_train_photometric``), still capturable.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import _lib, raster


class Tracker:
    def __init__(self, scene: raster.DeviceScene, intr, params: Optional[raster.Params] = None,
                 lr_trans: float = 0.001, lr_rot: float = 0.003, iters: int = 100, capacity_slack: float = 2.0,
                 schedule=None, w_ssim: float = 0.0):
        self.rast = raster.Rasterizer(scene, [intr], params or raster.Params())
        self.rast.schedule = schedule            # tile schedule of the fused kernel (autotuner's choice)
        self.lr_t, self.lr_r, self.iters = lr_trans, lr_rot, iters
        self.slack = capacity_slack
        P = self.rast.total_pixels
        self.pose = torch.zeros(12, device="cuda")
        self.grad_pose = torch.zeros(6, device="cuda")
        self.loss = torch.zeros(1, device="cuda")
        self.loss_hist = torch.zeros(iters, device="cuda")
        self.target_color = torch.zeros(3 * P, device="cuda")
        self.target_depth = torch.zeros(P, device="cuda")
        self.w_ssim = float(w_ssim)
        if self.w_ssim > 0:
            self.color = torch.empty(3 * P, device="cuda")
            self.depth = torch.empty(P, device="cuda")
            self.rast.photometric_scratch()      # allocated before any capture
        self.graph: Optional[torch.cuda.CUDAGraph] = None

    def set_frame(self, pose0: torch.Tensor, target_color: torch.Tensor, target_depth: torch.Tensor) -> None:
        """Load the initial pose and the observed frame (copied into the captured buffers).
        Grows the workspace when the new frame needs more pair capacity; a captured graph
        refers to the old workspace, so it is then dropped and must be captured again."""
        self.pose.copy_(pose0.reshape(12))
        self.target_color.copy_(target_color.reshape(-1))
        self.target_depth.copy_(target_depth.reshape(-1))
        k = self.rast.count(self.pose.view(1, 12))
        need = int(k * self.slack) + 8192
        if need > self.rast.capacity:
            self.rast.ensure_capacity(need)
            self.graph = None

    def _iteration(self, i: int) -> None:
        p = self.pose.view(1, 12)
        self.rast.bin_and_sort(p, check_capacity=False)
        if self.w_ssim > 0:
            self.rast.train_photometric(p, self.target_color, self.target_depth, w_ssim=self.w_ssim,
                                        color=self.color, depth=self.depth, loss=self.loss,
                                        out=(None, None, None, self.grad_pose))
        else:
            self.rast.train_l1(p, self.target_color, self.target_depth, loss=self.loss,
                               out=(None, None, None, self.grad_pose))
        self.rast.pose_step(p, self.grad_pose, self.lr_t, self.lr_r)
        self.loss_hist[i:i + 1].copy_(self.loss)

    def run_eager(self) -> torch.Tensor:
        for i in range(self.iters):
            self._iteration(i)
        return self.pose

    def capture(self) -> None:
        """Record `iters` iterations into one graph (the pose buffer is updated in place)."""
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                for i in range(self.iters):
                    self._iteration(i)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = g

    def replay(self) -> torch.Tensor:
        assert self.graph is not None, "capture() first"
        self.graph.replay()
        return self.pose

    def check(self) -> None:
        """Raise if any binning of the last run overflowed the workspace capacity."""
        _lib.check(self.rast.lib.tsr_check(raster._ptr(self.rast.ws), raster._stream(), None), "tsr_check")
