"""Mapping window: several keyframes rendered and back-propagated together (Sec. 3.4,
mapping re-renders a window of keyframes and optimises the map and their poses).

All views go through one projection/binning call (view id in the tile id), and one fused
forward + L1 + backward launch over every (view, tile) of the window, in the tile schedule the
autotuner picked for this workload (persistent workgroups pulling tiles from a device queue,
longest tile lists first, or one workgroup per tile).  Face gradients are summed across views
in the per-face accumulators; each view keeps its own pose gradient.  With ``w_ssim > 0`` the
step uses the full loss with the D-SSIM term (``tsr_render_train_photometric``; forward and
backward are then separate passes and the tile schedule is the default one).
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import autotune, raster


class MappingWindow:
    def __init__(self, scene: raster.DeviceScene, intrs: Sequence, params: Optional[raster.Params] = None,
                 schedule=None, table: Optional[str] = None, w_ssim: float = 0.0):
        self.rast = raster.Rasterizer(scene, intrs, params or raster.Params())
        self.n_views = len(intrs)
        self.intrs = list(intrs)
        self._schedule = schedule
        self._table = table
        P = self.rast.total_pixels
        self.color = torch.empty(3 * P, device="cuda")
        self.depth = torch.empty(P, device="cuda")
        self.loss = torch.zeros(self.n_views, device="cuda")
        self.grads = self.rast.grad_buffers()
        self.w_ssim = float(w_ssim)

    def prepare(self, poses: torch.Tensor, slack: float = 1.5) -> int:
        """Size the workspace and pick the schedule (table lookup) for these poses."""
        k = self.rast.fit(poses, slack)
        if self._schedule is None:
            self._schedule = autotune.lookup(self.intrs, k, self._table)
        self.rast.schedule = self._schedule
        return k

    @property
    def schedule(self):
        return self._schedule

    def step(self, poses: torch.Tensor, target_color: torch.Tensor, target_depth: torch.Tensor,
             check_capacity: bool = False):
        """One window iteration; returns (grad_pos, grad_col, grad_opa, grad_pose[V*6])."""
        self.rast.bin_and_sort(poses, check_capacity=check_capacity)
        if self.w_ssim > 0:
            return self.rast.train_photometric(poses, target_color, target_depth, w_ssim=self.w_ssim,
                                               color=self.color, depth=self.depth, loss=self.loss, out=self.grads)
        return self.rast.train_l1(poses, target_color, target_depth, color=self.color, depth=self.depth,
                                  loss=self.loss, out=self.grads)
