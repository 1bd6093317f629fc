"""One training iteration of R^2-Gaussian's hot path on the GPU.

Eq. 8: L = L1(I_r, I_m) + lambda_ssim D-SSIM(I_r, I_m) + lambda_tv TV(V_tv),
with I_r the projections of all views rendered in one launch (Sec. 3.2.1) and
V_tv a D^3 block voxelized at the target spacing (Sec. 3.2.2, Sec. 3.3).
Forward and backward of both operators and of the loss terms run in libgs.so;
the gradients of the two operators are summed into one set of parameter
gradients (the voxelizer backward accumulates onto the projection backward).
"""
from __future__ import annotations

import torch

from . import ops


class TrainingIteration:
    def __init__(self, mean, scale, quat, density, views: ops.Views, measured, block_shape,
                 lambda_ssim=0.25, lambda_tv=0.05, cutoff=3.0):
        self.params = (mean, scale, quat, density)
        self.views = views
        self.measured = measured
        self.lambda_ssim = float(lambda_ssim)
        self.lambda_tv = float(lambda_tv)
        self.cutoff = float(cutoff)
        dev = mean.device
        nz, ny, nx = block_shape
        f32 = dict(device=dev, dtype=torch.float32)
        self.image = torch.empty((views.n, views.height, views.width), **f32)
        self.grad_image = torch.empty_like(self.image)
        self.volume = torch.empty((nz, ny, nx), **f32)
        self.grad_volume = torch.empty_like(self.volume)
        self.loss_img = torch.empty(3, **f32)
        self.loss_tv = torch.empty(1, **f32)
        self.grads = tuple(torch.empty_like(p) for p in self.params)
        self.plan_proj = ops.Plan()
        self.plan_vox = ops.Plan()
        self.plan_loss = ops.Plan()

    def step(self, grid):
        """Forward + backward of the whole iteration; `grid` is the TV block's
        gs_grid (its origin changes from one iteration to the next)."""
        p = self.params
        ops.project_forward(*p, self.views, self.cutoff, self.plan_proj, out=self.image)
        ops.image_loss(self.image, self.measured, self.plan_loss, self.lambda_ssim,
                       loss_out=self.loss_img, grad_out=self.grad_image)
        ops.voxelize_forward(*p, grid, self.cutoff, self.plan_vox, out=self.volume)
        ops.tv_loss(self.volume, self.plan_loss, self.lambda_tv, loss_out=self.loss_tv,
                    grad_out=self.grad_volume)
        ops.project_backward(*p, self.views, self.grad_image, self.plan_proj, self.cutoff,
                             grads=self.grads, accumulate=False)
        ops.voxelize_backward(*p, grid, self.grad_volume, self.plan_vox, self.cutoff,
                              grads=self.grads, accumulate=True)
        return self.grads

    def total_loss(self):
        """L1 + lambda_ssim (1 - SSIM) + lambda_tv TV, as a device scalar."""
        return self.loss_img[0] + self.lambda_tv * self.loss_tv[0]
