"""PyTorch-facing wrappers of include/gs_train.h: densification statistics,
Adam, adaptive density control, volume metrics and the trainer.  Argument
marshalling only; every computation runs in libgs.so."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _native as N
from .ops import Views, _dev, _gaussians, _grads, _stream, grid_from, Plan

# (name, components per Gaussian) of the gs_params arrays
PARAM_LAYOUT = (("mean", 3), ("log_scale", 3), ("quat", 4), ("density_raw", 1), ("scale", 3),
                ("density", 1), ("m_mean", 3), ("m_scale", 3), ("m_quat", 4), ("m_density", 1),
                ("v_mean", 3), ("v_scale", 3), ("v_quat", 4), ("v_density", 1))


def _shape(cap, k):
    return (cap,) if k == 1 else (cap, k)


class ParamState:
    """Trainable state (gs_params) in torch tensors of a fixed capacity."""

    def __init__(self, capacity, device="cuda"):
        self.capacity = int(capacity)
        self.t = {name: torch.zeros(_shape(self.capacity, k), device=device, dtype=torch.float32)
                  for name, k in PARAM_LAYOUT}

    @classmethod
    def from_activated(cls, mean, scale, quat, density, capacity=None):
        n = density.shape[0]
        st = cls(capacity or n, mean.device)
        st.t["mean"][:n] = mean
        st.t["scale"][:n] = scale
        st.t["quat"][:n] = quat
        st.t["density"][:n] = density
        N.call("gs_params_from_activated", ctypes.byref(st.struct()), n, _stream())
        return st

    def struct(self):
        p = N.GsParams()
        for name, _ in PARAM_LAYOUT:
            setattr(p, name, _dev(self.t[name], name))
        return p

    def activated(self, n):
        return tuple(self.t[k][:n] for k in ("mean", "scale", "quat", "density"))


def project_backward_stats(mean, scale, quat, density, views: Views, grad_image, plan, grad_sum,
                           visible, stat_scale=1.0, cutoff=3.0, grads=None, accumulate=False):
    g = _gaussians(mean, scale, quat, density)
    if grads is None:
        grads = tuple(torch.empty_like(t) for t in (mean, scale, quat, density))
    gr = _grads(*grads)
    if visible.dtype != torch.int32 or not visible.is_cuda or not visible.is_contiguous():
        raise ValueError("visible must be a contiguous int32 tensor on the GPU")
    st = N.GsGradStats(_dev(grad_sum, "grad_sum", (g.n,)), ctypes.c_void_p(visible.data_ptr()),
                       float(stat_scale))
    N.call("gs_project_bwd_stats", ctypes.byref(g), views.arr, views.n, float(cutoff),
           _dev(grad_image, "grad_image", (views.n, views.height, views.width)), ctypes.byref(gr),
           int(bool(accumulate)), ctypes.byref(st), plan.handle, _stream())
    return grads


def random_normals(seed, counter, n, out=None):
    """n standard normal draws (Philox4x32-10 + Box-Muller) on the device."""
    if out is None:
        out = torch.empty(max(int(n), 1), device="cuda", dtype=torch.float32)
    N.call("gs_random_normals", int(seed) & 0xFFFFFFFFFFFFFFFF, int(counter) & 0xFFFFFFFFFFFFFFFF,
           int(n), _dev(out, "out"), _stream())
    return out[:int(n)]


def adam_step(state: ParamState, n, grads, lrs, step):
    """grads: (mean, scale, quat, density) gradients w.r.t. the activated
    parameters; lrs: dict with keys mean, scale, quat, density."""
    cfg = N.GsAdamConfig(float(lrs["mean"]), float(lrs["scale"]), float(lrs["quat"]),
                         float(lrs["density"]), int(step))
    N.call("gs_adam_step", ctypes.byref(state.struct()), int(n), ctypes.byref(_grads(*grads)),
           ctypes.byref(cfg), _stream())


def densify(src: ParamState, n, grad_sum, visible, normals, grad_threshold, clone_max_scale,
            min_density, densify=True, dst_capacity=None, plan=None):
    """Adaptive density control; returns (dst ParamState, new count, action
    tensor [n])."""
    plan = plan or Plan()
    cap = int(dst_capacity or max(2 * n, 1))
    dst = ParamState(cap, src.t["mean"].device)
    action = torch.empty(max(n, 1), device=src.t["mean"].device, dtype=torch.int32)
    st = N.GsGradStats(ctypes.c_void_p(grad_sum.data_ptr()), ctypes.c_void_p(visible.data_ptr()), 1.0)
    cfg = N.GsDensifyConfig(float(grad_threshold), float(clone_max_scale), float(min_density),
                            int(bool(densify)))
    n_out = ctypes.c_int64()
    nrm = None if normals is None else _dev(normals, "normals", (n, 2, 3))
    N.call("gs_densify", ctypes.byref(src.struct()), int(n), ctypes.byref(st), nrm,
           ctypes.byref(cfg), ctypes.byref(dst.struct()), cap, ctypes.c_void_p(action.data_ptr()),
           ctypes.byref(n_out), plan.handle, _stream())
    return dst, n_out.value, action[:n]


def volume_metrics(volume, gt, plan=None):
    """(PSNR, SSIM) of a [nz][ny][nx] volume against the ground truth."""
    nz, ny, nx = gt.shape
    ps, ss = ctypes.c_double(), ctypes.c_double()
    plan = plan or Plan()  # held until the call returns (its __del__ frees the plan)
    N.call("gs_volume_metrics", _dev(volume, "volume", (nz, ny, nx)), _dev(gt, "gt", (nz, ny, nx)),
           nx, ny, nz, ctypes.byref(ps), ctypes.byref(ss), plan.handle, _stream())
    return ps.value, ss.value


def train_config(**overrides):
    """gs_train_config with the defaults of the paper (Sec. 4.1), updated by
    keyword arguments named like its fields."""
    c = N.GsTrainConfig()
    N.lib().gs_train_config_default(ctypes.byref(c))
    for k, v in overrides.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


class Trainer:
    """The optimisation loop (gs_trainer) on its own stream."""

    def __init__(self, mean, scale, quat, density, measured, views: Views, grid, **config):
        self.config = train_config(**config)
        g = _gaussians(mean, scale, quat, density)
        n_views = views.n
        _dev(measured, "measured", (n_views, views.height, views.width))
        self._measured = measured  # the trainer keeps the pointer
        self._views = views
        self._grid = grid_from(grid) if not isinstance(grid, N.GsGrid) else grid
        torch.cuda.synchronize()  # inputs come from torch's stream
        h = ctypes.c_void_p()
        N.call("gs_trainer_create", ctypes.byref(self.config), ctypes.byref(g),
               ctypes.c_void_p(measured.data_ptr()), views.arr, n_views, ctypes.byref(self._grid),
               ctypes.byref(h))
        self._h = h

    def run(self, iters):
        losses = np.zeros(max(int(iters), 1), np.float32)
        N.call("gs_trainer_run", self._h, int(iters), losses.ctypes.data_as(ctypes.c_void_p))
        return losses[:int(iters)]

    def step(self, view_idx, tv_offset=(0, 0, 0), normals=None):
        vi = (ctypes.c_int32 * len(view_idx))(*[int(v) for v in view_idx])
        off = (ctypes.c_int32 * 3)(*[int(v) for v in tv_offset])
        if normals is not None:
            torch.cuda.synchronize()
        loss = ctypes.c_float()
        N.call("gs_trainer_step", self._h, vi, off,
               None if normals is None else ctypes.c_void_p(normals.data_ptr()), ctypes.byref(loss))
        return loss.value

    def count(self):
        n = ctypes.c_int64()
        N.call("gs_trainer_state", self._h, None, ctypes.byref(n), None)
        return n.value

    def model(self):
        """Copies of the current activated parameters (mean, scale, quat, density)."""
        n = self.count()
        out = [torch.empty(_shape(max(n, 1), k), device="cuda") for k in (3, 3, 4, 1)]
        torch.cuda.synchronize()
        got = ctypes.c_int64()
        N.call("gs_trainer_export", self._h, max(n, 1), *[ctypes.c_void_p(t.data_ptr()) for t in out],
               ctypes.byref(got))
        return tuple(t[:got.value] for t in out)

    def iteration(self):
        g, it = N.GsGaussians(), ctypes.c_int32()
        N.call("gs_trainer_model", self._h, ctypes.byref(g), ctypes.byref(it))
        return it.value

    def evaluate(self, grid, gt=None):
        """Voxelized model on grid (X-3DGS: densities corrected by the mean
        rectification factor first) and, with gt, (PSNR, SSIM)."""
        gg = grid_from(grid) if not isinstance(grid, N.GsGrid) else grid
        vol = torch.empty((gg.nz, gg.ny, gg.nx), device="cuda")
        ps, ss = ctypes.c_double(), ctypes.c_double()
        torch.cuda.synchronize()
        N.call("gs_trainer_evaluate", self._h, ctypes.byref(gg), ctypes.c_void_p(vol.data_ptr()),
               None if gt is None else _dev(gt, "gt", (gg.nz, gg.ny, gg.nx)),
               ctypes.byref(ps), ctypes.byref(ss))
        return vol, (ps.value, ss.value) if gt is not None else None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            N.lib().gs_trainer_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
