"""PyTorch-facing entry points of the HIP path.

Every computation runs in libgs.so; this module only checks tensor
properties, marshals pointers and the current HIP stream, and wraps the
forward/backward pairs as ``torch.autograd.Function``s.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _native as N


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, name, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 tensor on the GPU")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _ptr_or_null(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Plan:
    """Workspace and saved forward state of the library (gs_plan)."""

    def __init__(self):
        h = ctypes.c_void_p()
        N.call("gs_plan_create", None, None, None, ctypes.byref(h))
        self._h = h

    @property
    def handle(self):
        return self._h

    def status(self):
        sk, en = ctypes.c_int64(), ctypes.c_int64()
        N.call("gs_plan_status", self._h, ctypes.byref(sk), ctypes.byref(en))
        return {"skipped": sk.value, "tile_entries": en.value}

    def reserve(self, max_gaussians, max_views=0, width=0, height=0, max_proj_entries=0,
                grid=(0, 0, 0), max_vox_entries=0, max_tv_voxels=0, max_records=0,
                forward_only=False):
        """Allocate for problems up to these sizes and stop allocating and
        synchronizing in operator calls (gs_plan_reserve)."""
        r = N.GsReserve(int(max_gaussians), int(max_views), int(width), int(height),
                        int(max_proj_entries), int(grid[0]), int(grid[1]), int(grid[2]),
                        int(max_vox_entries), int(max_tv_voxels), int(max_records),
                        int(bool(forward_only)))
        N.call("gs_plan_reserve", self._h, ctypes.byref(r), _stream())

    def check(self, raise_overflow=True):
        """(largest projection entries, largest voxel entries) since the last
        check; if a call exceeded the reservation, raises GsError
        (GS_EOVERFLOW), or with raise_overflow=False returns the counts and
        True as a third item (the record is cleared either way)."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        st = N.lib().gs_plan_check(self._h, ctypes.byref(a), ctypes.byref(b))
        if st == 3 and not raise_overflow:
            return a.value, b.value, True
        if st != 0:
            raise N.GsError("gs_plan_check", st, N.lib().gs_last_error().decode(errors="replace"))
        return (a.value, b.value) if raise_overflow else (a.value, b.value, False)

    def set_rectify(self, enable=True):
        """False: unrectified (3DGS-style) projection rho_hat = rho."""
        N.call("gs_plan_set_rectify", self._h, int(bool(enable)))

    def set_timing(self, enable=True):
        N.call("gs_plan_set_timing", self._h, int(bool(enable)))

    def stage_times(self):
        """{stage: (total ms, launches)} since the previous query."""
        n = len(N.STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        N.call("gs_plan_stage_times", self._h, ms, cnt, n)
        return {N.STAGES[i]: (ms[i], cnt[i]) for i in range(n) if cnt[i]}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            N.lib().gs_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Views:
    """A host array of gs_view (all views share the detector size)."""

    def __init__(self, arr):
        self.arr = arr
        self.n = len(arr)
        self.width = arr[0].width
        self.height = arr[0].height

    @classmethod
    def cone(cls, thetas, src_obj, src_det, width, height, pitch):
        thetas = list(np.asarray(thetas, np.float64).reshape(-1))
        arr = (N.GsView * len(thetas))()
        for i, th in enumerate(thetas):
            N.call("gs_view_cone", float(th), float(src_obj), float(src_det), int(width),
                   int(height), float(pitch), ctypes.byref(arr[i]))
        return cls(arr)

    @classmethod
    def parallel(cls, rots, width, height, pitch, off_u=0.0, off_v=0.0):
        rots = np.asarray(rots, np.float64).reshape(-1, 3, 3)
        arr = (N.GsView * len(rots))()
        for i, R in enumerate(rots):
            v = arr[i]
            v.beam = N.GS_PARALLEL
            v.width, v.height = int(width), int(height)
            v.pitch_u = v.pitch_v = float(pitch)
            v.off_u, v.off_v = float(off_u), float(off_v)
            for k, x in enumerate(R.reshape(-1)):
                v.rot[k] = float(x)
        return cls(arr)

    @classmethod
    def from_scan(cls, scan):
        if hasattr(scan, "thetas"):
            return cls.cone(scan.thetas, scan.src_obj, scan.src_det, scan.width, scan.height,
                            scan.pitch)
        return cls.parallel(scan.rots, scan.width, scan.height, scan.pitch)

    def subset(self, idx):
        idx = list(idx)
        arr = (N.GsView * len(idx))()
        for j, i in enumerate(idx):
            ctypes.memmove(ctypes.byref(arr[j]), ctypes.byref(self.arr[i]), ctypes.sizeof(N.GsView))
        return Views(arr)


def make_grid(nx, ny, nz, origin, spacing):
    g = N.GsGrid()
    g.nx, g.ny, g.nz = int(nx), int(ny), int(nz)
    for k in range(3):
        g.origin[k] = float(origin[k])
        g.spacing[k] = float(spacing[k])
    return g


def grid_from(grid):
    return make_grid(grid.nx, grid.ny, grid.nz, grid.origin, grid.spacing)


def _gaussians(mean, scale, quat, density):
    n = density.shape[0] if density.dim() == 1 else -1
    g = N.GsGaussians()
    g.n = n
    g.mean = _dev(mean, "mean", (n, 3))
    g.scale = _dev(scale, "scale", (n, 3))
    g.quat = _dev(quat, "quat", (n, 4))
    g.density = _dev(density, "density", (n,))
    return g


def _grads(gm, gs, gq, gd):
    r = N.GsGrads()
    r.mean, r.scale, r.quat, r.density = (_ptr_or_null(t) for t in (gm, gs, gq, gd))
    return r


# ------------------------------------------------------------------ calls --

def project_forward(mean, scale, quat, density, views: Views, cutoff=3.0, plan=None, out=None):
    g = _gaussians(mean, scale, quat, density)
    if out is None:
        out = torch.empty((views.n, views.height, views.width), device=mean.device,
                          dtype=torch.float32)
    N.call("gs_project_fwd", ctypes.byref(g), views.arr, views.n, float(cutoff),
           _dev(out, "image", (views.n, views.height, views.width)),
           plan.handle if plan is not None else None, _stream())
    return out


def project_forward_multi(models, view_model, views: Views, cutoff=3.0, plan=None, out=None):
    """Views of several Gaussian sets in one launch (gs_project_fwd_multi):
    view v renders models[view_model[v]], each model a (mean, scale, quat,
    density) tuple of tensors.  Returns the image stack [V, H, W]."""
    arr = (N.GsGaussians * len(models))()
    for i, m in enumerate(models):
        arr[i] = _gaussians(*m)
    vm = (ctypes.c_int32 * views.n)(*[int(x) for x in view_model])
    dev = models[0][0].device
    if out is None:
        out = torch.empty((views.n, views.height, views.width), device=dev, dtype=torch.float32)
    keep = plan if plan is not None else Plan()  # held until the call returns
    N.call("gs_project_fwd_multi", arr, len(models), vm, views.arr, views.n, float(cutoff),
           _dev(out, "out", (views.n, views.height, views.width)), keep.handle, _stream())
    return out


def project_backward(mean, scale, quat, density, views: Views, grad_image, plan, cutoff=3.0,
                     grads=None, accumulate=False):
    g = _gaussians(mean, scale, quat, density)
    if grads is None:
        grads = tuple(torch.empty_like(t) for t in (mean, scale, quat, density))
    for t, name in zip(grads, ("mean", "scale", "quat", "density")):
        if t is not None:
            _dev(t, "grad_" + name)
    gr = _grads(*grads)
    N.call("gs_project_bwd", ctypes.byref(g), views.arr, views.n, float(cutoff),
           _dev(grad_image, "grad_image", (views.n, views.height, views.width)), ctypes.byref(gr),
           int(bool(accumulate)), plan.handle, _stream())
    return grads


def mean_mu(mean, scale, quat, density, views: Views, plan=None):
    """Per-Gaussian mean rectification factor over the views, and the density
    divided by it (what the unrectified X-3DGS variant voxelizes)."""
    g = _gaussians(mean, scale, quat, density)
    mu = torch.empty_like(density)
    dens = torch.empty_like(density)
    plan = plan or Plan()  # held until the call returns (its __del__ frees the plan)
    N.call("gs_project_mean_mu", ctypes.byref(g), views.arr, views.n, _dev(mu, "mu_out"),
           _dev(dens, "density_out"), plan.handle, _stream())
    return mu, dens


def voxelize_forward(mean, scale, quat, density, grid, cutoff=3.0, plan=None, out=None):
    g = _gaussians(mean, scale, quat, density)
    if out is None:
        out = torch.empty((grid.nz, grid.ny, grid.nx), device=mean.device, dtype=torch.float32)
    N.call("gs_voxelize_fwd", ctypes.byref(g), ctypes.byref(grid), float(cutoff),
           _dev(out, "volume", (grid.nz, grid.ny, grid.nx)),
           plan.handle if plan is not None else None, _stream())
    return out


def voxelize_backward(mean, scale, quat, density, grid, grad_volume, plan, cutoff=3.0, grads=None,
                      accumulate=False):
    g = _gaussians(mean, scale, quat, density)
    if grads is None:
        grads = tuple(torch.empty_like(t) for t in (mean, scale, quat, density))
    gr = _grads(*grads)
    N.call("gs_voxelize_bwd", ctypes.byref(g), ctypes.byref(grid), float(cutoff),
           _dev(grad_volume, "grad_volume", (grid.nz, grid.ny, grid.nx)), ctypes.byref(gr),
           int(bool(accumulate)), plan.handle, _stream())
    return grads


def image_loss(render, measured, plan, lambda_ssim=0.25, grad=True, loss_out=None, grad_out=None):
    """Returns (loss tensor [3] = total, l1, ssim; grad of total w.r.t. render or None)."""
    n, h, w = render.shape
    if loss_out is None:
        loss_out = torch.empty(3, device=render.device, dtype=torch.float32)
    if grad and grad_out is None:
        grad_out = torch.empty_like(render)
    N.call("gs_loss_image", _dev(render, "render"), _dev(measured, "measured", (n, h, w)), n, h, w,
           float(lambda_ssim), _dev(loss_out, "loss_out", (3,)),
           _dev(grad_out, "grad", (n, h, w)) if grad else None, plan.handle, _stream())
    return loss_out, (grad_out if grad else None)


def image_loss_noalloc(render, measured, lambda_ssim=0.25, grad=True, loss_out=None,
                       grad_out=None):
    """image_loss through gs_loss_image_noalloc: no plan, and the library
    allocates nothing (its partial sums live in a static per-GPU buffer)."""
    n, h, w = render.shape
    if loss_out is None:
        loss_out = torch.empty(3, device=render.device, dtype=torch.float32)
    if grad and grad_out is None:
        grad_out = torch.empty_like(render)
    N.call("gs_loss_image_noalloc", _dev(render, "render"), _dev(measured, "measured", (n, h, w)),
           n, h, w, float(lambda_ssim), _dev(loss_out, "loss_out", (3,)),
           _dev(grad_out, "grad_out", (n, h, w)) if grad else None, _stream())
    return loss_out, (grad_out if grad else None)


def tv_loss(volume, plan, weight=1.0, grad=True, accumulate=False, loss_out=None, grad_out=None):
    nz, ny, nx = volume.shape
    if loss_out is None:
        loss_out = torch.empty(1, device=volume.device, dtype=torch.float32)
    if grad and grad_out is None:
        grad_out = torch.empty_like(volume)
    N.call("gs_loss_tv", _dev(volume, "volume"), nx, ny, nz, float(weight),
           _dev(loss_out, "loss_out", (1,)), _dev(grad_out, "grad", (nz, ny, nx)) if grad else None,
           int(bool(accumulate)), plan.handle, _stream())
    return loss_out, (grad_out if grad else None)


# -------------------------------------------------------------- autograd --

class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean, scale, quat, density, views, cutoff, plan):
        img = project_forward(mean, scale, quat, density, views, cutoff, plan)
        ctx.save_for_backward(mean, scale, quat, density)
        ctx.views, ctx.cutoff, ctx.plan = views, cutoff, plan
        return img

    @staticmethod
    def backward(ctx, grad_image):
        mean, scale, quat, density = ctx.saved_tensors
        need = ctx.needs_input_grad[:4]
        grads = tuple(torch.empty_like(t) if nd else None
                      for t, nd in zip((mean, scale, quat, density), need))
        project_backward(mean, scale, quat, density, ctx.views, grad_image.contiguous(), ctx.plan,
                         ctx.cutoff, grads)
        return (*grads, None, None, None)


class _Voxelize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean, scale, quat, density, grid, cutoff, plan):
        vol = voxelize_forward(mean, scale, quat, density, grid, cutoff, plan)
        ctx.save_for_backward(mean, scale, quat, density)
        ctx.grid, ctx.cutoff, ctx.plan = grid, cutoff, plan
        return vol

    @staticmethod
    def backward(ctx, grad_volume):
        mean, scale, quat, density = ctx.saved_tensors
        need = ctx.needs_input_grad[:4]
        grads = tuple(torch.empty_like(t) if nd else None
                      for t, nd in zip((mean, scale, quat, density), need))
        voxelize_backward(mean, scale, quat, density, ctx.grid, grad_volume.contiguous(), ctx.plan,
                          ctx.cutoff, grads)
        return (*grads, None, None, None)


def project(mean, scale, quat, density, views: Views, cutoff=3.0, plan=None):
    """Differentiable X-ray projection [V, H, W] (HIP forward and backward)."""
    return _Project.apply(mean, scale, quat, density, views, cutoff, plan or Plan())


def voxelize(mean, scale, quat, density, grid, cutoff=3.0, plan=None):
    """Differentiable voxelization [nz, ny, nx] (HIP forward and backward)."""
    return _Voxelize.apply(mean, scale, quat, density, grid, cutoff, plan or Plan())


# ---------------------------------------------------------------- serving --

class Server:
    """Request loop of include/gs_serve.h: worker threads with their own
    streams and plans; continuous batching of projections across models into
    one launch within reserved workspaces sized from the HBM budget (with
    graphs=True each batch replays a HIP graph captured for its shape), or the
    plain one-request-per-launch path.  All work runs in libgs.so."""

    def __init__(self, n_workers=4, batching=True, max_batch_views=128, cutoff=3.0,
                 hbm_budget_bytes=None, graphs=False):
        if hbm_budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget_bytes = int(0.25 * free)
        mode = (2 if graphs else 1) if batching else 0
        cfg = N.GsServerConfig(int(n_workers), mode, int(max_batch_views),
                               float(cutoff), int(hbm_budget_bytes))
        h = ctypes.c_void_p()
        N.call("gs_server_create", ctypes.byref(cfg), ctypes.byref(h))
        self._h = h
        self._models = []

    def reserved_bytes(self):
        """Device bytes the workers reserved for the last continuous run."""
        b = ctypes.c_int64()
        N.call("gs_server_reserved_bytes", self._h, ctypes.byref(b))
        return b.value

    def add_model(self, mean, scale, quat, density):
        g = _gaussians(mean, scale, quat, density)
        mid = ctypes.c_int32()
        N.call("gs_server_add_model", self._h, ctypes.byref(g), ctypes.byref(mid))
        self._models.append((mean, scale, quat, density))  # keep the tensors alive
        return mid.value

    def run(self, requests, time_scale=1.0):
        """requests: list of dicts with kind ('project' | 'volume'), model,
        arrival_s, and views (Views) or grid (gs_grid), optional out tensor.
        Returns (list of result dicts, wall seconds)."""
        n = len(requests)
        arr = (N.GsRequest * n)()
        keep = []
        for i, r in enumerate(requests):
            q = arr[i]
            q.model = int(r["model"])
            q.arrival_s = float(r["arrival_s"])
            out = r.get("out")
            if r["kind"] == "project":
                q.kind = 0
                q.n_views = r["views"].n
                q.views = ctypes.cast(r["views"].arr, ctypes.POINTER(N.GsView))
                keep.append(r["views"])
                if out is not None:
                    _dev(out, "out", (r["views"].n, r["views"].height, r["views"].width))
            else:
                q.kind = 1
                q.grid = r["grid"]
                if out is not None:
                    _dev(out, "out", (r["grid"].nz, r["grid"].ny, r["grid"].nx))
            q.out = _ptr_or_null(out)
        res = (N.GsRequestResult * n)()
        wall = ctypes.c_double()
        N.call("gs_server_run", self._h, arr, n, float(time_scale), res, ctypes.byref(wall))
        out = [{"start_s": x.start_s, "done_s": x.done_s, "latency_s": x.latency_s,
                "batch_size": x.batch_size, "status": x.status} for x in res]
        return out, wall.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            N.lib().gs_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
