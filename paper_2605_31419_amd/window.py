"""Mapping window: several keyframes rendered and back-propagated together (Sec. 3.4,
mapping re-renders a window of keyframes and optimises the map and their poses).

All views go through one projection/binning call (view id in the tile id), and one fused
forward + L1 + backward launch over every (view, tile) of the window, in the tile schedule the
autotuner picked for this workload (persistent workgroups pulling tiles from a device queue,
longest tile lists first, or one workgroup per tile).  Face gradients are summed across views
in the per-face accumulators; each view keeps its own pose gradient.  With ``w_ssim > 0`` the
step uses the full loss with the D-SSIM term (``tsr_render_train_photometric``; forward and
backward are then separate passes and the tile schedule is the default one).  ``w_equi`` adds
the equilateral regulariser (eq. 14) and ``w_norm`` the normal loss against per-view target
normals, both accumulated on the device into the same gradient buffers, giving the mapping
energy E_pho + lambda_dep E_dep + lambda_norm E_norm + lambda_equi E_equi.  With the normal
loss the step is ``tsr_render_train_mapping``: one binning, one forward that composites the
face normals as three more channels, one backward that takes the colour, depth and normal
seeds.  ``fused_mapping=False`` runs the normal loss as its own step instead (a second
workspace binned with the face normals as colours), the slower form kept for comparison.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import autotune, raster


class MappingWindow:
    def __init__(self, scene: raster.DeviceScene, intrs: Sequence, params: Optional[raster.Params] = None,
                 schedule=None, table: Optional[str] = None, w_ssim: float = 0.0, w_equi: float = 0.0,
                 w_norm: float = 0.0, fused_mapping: bool = True):
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
        self.w_equi = float(w_equi)
        self.w_norm = float(w_norm)
        self.equi_loss = torch.zeros(1, device="cuda")
        self.norm_loss = torch.zeros(self.n_views, device="cuda")
        self.fused_mapping = bool(fused_mapping)
        self.normal_map: Optional[torch.Tensor] = None
        self.nrast = (raster.Rasterizer(scene, intrs, params or raster.Params())
                      if self.w_norm > 0 and not self.fused_mapping else None)

    def prepare(self, poses: torch.Tensor, slack: float = 1.5) -> int:
        """Size the workspace and pick the schedule (table lookup) for these poses."""
        k = self.rast.fit(poses, slack)
        if self.nrast is not None:
            self.nrast.fit(poses, slack)
        if self._schedule is None:
            self._schedule = autotune.lookup(self.intrs, k, self._table)
        self.rast.schedule = self._schedule
        return k

    @property
    def schedule(self):
        return self._schedule

    def step(self, poses: torch.Tensor, target_color: torch.Tensor, target_depth: torch.Tensor,
             check_capacity: bool = False, target_normals: Optional[torch.Tensor] = None):
        """One window iteration; returns (grad_pos, grad_col, grad_opa, grad_pose[V*6])."""
        self.rast.bin_and_sort(poses, check_capacity=check_capacity)
        if self.w_norm > 0 and self.fused_mapping and target_normals is not None:
            self.rast.train_mapping(poses, target_color, target_depth, target_normals, w_ssim=self.w_ssim,
                                    w_norm=self.w_norm, color=self.color, depth=self.depth,
                                    normal_map=self.normal_map, loss=self.loss, loss_norm=self.norm_loss,
                                    out=self.grads)
            if self.w_equi > 0:
                raster.equilateral(self.rast.scene, weight=self.w_equi, grad=self.grads[0], accumulate=True,
                                   loss=self.equi_loss)
            return self.grads
        if self.w_ssim > 0:
            self.rast.train_photometric(poses, target_color, target_depth, w_ssim=self.w_ssim,
                                        color=self.color, depth=self.depth, loss=self.loss, out=self.grads)
        else:
            self._train_l1(poses, target_color, target_depth)
        gp, _, go, gpose = self.grads
        if self.w_equi > 0:
            raster.equilateral(self.rast.scene, weight=self.w_equi, grad=gp, accumulate=True, loss=self.equi_loss)
        if self.nrast is not None and target_normals is not None:
            self.nrast.train_normal(poses, target_normals, w_norm=self.w_norm, loss=self.norm_loss,
                                    out=(gp, go, gpose), accumulate=True)
        return self.grads

    def _train_l1(self, poses, target_color, target_depth):
        return self.rast.train_l1(poses, target_color, target_depth, color=self.color, depth=self.depth,
                                  loss=self.loss, out=self.grads)
