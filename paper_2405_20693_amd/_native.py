"""ctypes view of libgs.so (include/gs.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgs.so")

c_int32, c_int64, c_float, c_double, c_void_p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                                 ctypes.c_double, ctypes.c_void_p)

STAGES = ("proj_bin", "proj_scatter", "render_fwd", "render_bwd", "proj_chain", "vox_bin",
          "vox_scatter", "vox_fwd", "vox_bwd", "vox_chain", "loss_image", "loss_tv")

GS_PARALLEL = 0
GS_CONE = 1

STATUS = {0: "GS_OK", 1: "GS_EINVAL", 2: "GS_ENOMEM", 3: "GS_EOVERFLOW", 4: "GS_EHIP",
          5: "GS_EUNSUPPORTED"}


class GsView(ctypes.Structure):
    _fields_ = [("beam", c_int32), ("width", c_int32), ("height", c_int32),
                ("pitch_u", c_float), ("pitch_v", c_float), ("off_u", c_float), ("off_v", c_float),
                ("rot", c_float * 9), ("src_obj", c_float), ("src_det", c_float)]


class GsGrid(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
                ("origin", c_float * 3), ("spacing", c_float * 3)]


class GsGaussians(ctypes.Structure):
    _fields_ = [("n", c_int64), ("mean", c_void_p), ("scale", c_void_p), ("quat", c_void_p),
                ("density", c_void_p)]


class GsGrads(ctypes.Structure):
    _fields_ = [("mean", c_void_p), ("scale", c_void_p), ("quat", c_void_p), ("density", c_void_p)]


class GsServerConfig(ctypes.Structure):
    _fields_ = [("n_workers", c_int32), ("batching", c_int32), ("max_batch_views", c_int32),
                ("cutoff", c_float), ("hbm_budget_bytes", c_int64)]


class GsRequest(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("model", c_int32), ("arrival_s", c_double),
                ("n_views", c_int32), ("views", ctypes.POINTER(GsView)), ("grid", GsGrid),
                ("out", c_void_p)]


class GsRequestResult(ctypes.Structure):
    _fields_ = [("start_s", c_double), ("done_s", c_double), ("latency_s", c_double),
                ("batch_size", c_int32), ("status", c_int32)]


class GsReserve(ctypes.Structure):
    _fields_ = [("max_gaussians", c_int64), ("max_views", c_int32), ("width", c_int32),
                ("height", c_int32), ("max_proj_entries", c_int64), ("nx", c_int32),
                ("ny", c_int32), ("nz", c_int32), ("max_vox_entries", c_int64),
                ("max_tv_voxels", c_int64), ("max_records", c_int64), ("forward_only", c_int32)]


class GsGradStats(ctypes.Structure):
    _fields_ = [("grad_sum", c_void_p), ("visible", c_void_p), ("scale", c_float)]


PARAM_FIELDS = ("mean", "log_scale", "quat", "density_raw", "scale", "density",
                "m_mean", "m_scale", "m_quat", "m_density", "v_mean", "v_scale", "v_quat",
                "v_density")


class GsParams(ctypes.Structure):
    _fields_ = [(f, c_void_p) for f in PARAM_FIELDS]


class GsAdamConfig(ctypes.Structure):
    _fields_ = [("lr_mean", c_float), ("lr_scale", c_float), ("lr_quat", c_float),
                ("lr_density", c_float), ("step", c_int32)]


class GsDensifyConfig(ctypes.Structure):
    _fields_ = [("grad_threshold", c_float), ("clone_max_scale", c_float),
                ("min_density", c_float), ("densify", c_int32)]


class GsTrainConfig(ctypes.Structure):
    _fields_ = [("iterations", c_int32), ("views_per_iter", c_int32),
                ("lr_mean", c_float), ("lr_density", c_float), ("lr_scale", c_float),
                ("lr_quat", c_float), ("lr_final_ratio", c_float), ("lambda_ssim", c_float),
                ("lambda_tv", c_float), ("tv_size", c_int32), ("densify_from", c_int32),
                ("densify_until", c_int32), ("densify_interval", c_int32),
                ("grad_threshold", c_float), ("clone_max_scale", c_float),
                ("min_density", c_float), ("cutoff", c_float), ("rectify", c_int32),
                ("seed", ctypes.c_uint64)]


class GsError(RuntimeError):
    def __init__(self, func, status, message):
        self.status = status
        super().__init__(f"{func}: {STATUS.get(status, status)}: {message}")


_lib = None

EXPORTS = {
    "gs_plan_create": (ctypes.c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_void_p)]),
    "gs_plan_destroy": (None, [c_void_p]),
    "gs_plan_status": (ctypes.c_int, [c_void_p, ctypes.POINTER(c_int64), ctypes.POINTER(c_int64)]),
    "gs_view_cone": (ctypes.c_int, [c_double, c_float, c_float, c_int32, c_int32, c_float,
                                    ctypes.POINTER(GsView)]),
    "gs_project_fwd": (ctypes.c_int, [ctypes.POINTER(GsGaussians), ctypes.POINTER(GsView), c_int32,
                                      c_float, c_void_p, c_void_p, c_void_p]),
    "gs_project_fwd_multi": (ctypes.c_int, [ctypes.POINTER(GsGaussians), c_int32,
                                            ctypes.POINTER(c_int32), ctypes.POINTER(GsView), c_int32,
                                            c_float, c_void_p, c_void_p, c_void_p]),
    "gs_project_bwd": (ctypes.c_int, [ctypes.POINTER(GsGaussians), ctypes.POINTER(GsView), c_int32,
                                      c_float, c_void_p, ctypes.POINTER(GsGrads), c_int32, c_void_p,
                                      c_void_p]),
    "gs_voxelize_fwd": (ctypes.c_int, [ctypes.POINTER(GsGaussians), ctypes.POINTER(GsGrid), c_float,
                                       c_void_p, c_void_p, c_void_p]),
    "gs_voxelize_bwd": (ctypes.c_int, [ctypes.POINTER(GsGaussians), ctypes.POINTER(GsGrid), c_float,
                                       c_void_p, ctypes.POINTER(GsGrads), c_int32, c_void_p,
                                       c_void_p]),
    "gs_loss_image": (ctypes.c_int, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_float,
                                     c_void_p, c_void_p, c_void_p, c_void_p]),
    "gs_loss_image_noalloc": (ctypes.c_int, [c_void_p, c_void_p, c_int32, c_int32, c_int32,
                                             c_float, c_void_p, c_void_p, c_void_p]),
    "gs_loss_tv": (ctypes.c_int, [c_void_p, c_int32, c_int32, c_int32, c_float, c_void_p, c_void_p,
                                  c_int32, c_void_p, c_void_p]),
    "gs_plan_set_timing": (ctypes.c_int, [c_void_p, c_int32]),
    "gs_plan_reserve": (ctypes.c_int, [c_void_p, ctypes.POINTER(GsReserve), c_void_p]),
    "gs_plan_reserve_bytes": (ctypes.c_int, [ctypes.POINTER(GsReserve), ctypes.POINTER(c_int64)]),
    "gs_plan_check": (ctypes.c_int, [c_void_p, ctypes.POINTER(c_int64), ctypes.POINTER(c_int64)]),
    "gs_plan_set_rectify": (ctypes.c_int, [c_void_p, c_int32]),
    "gs_project_mean_mu": (ctypes.c_int, [ctypes.POINTER(GsGaussians), ctypes.POINTER(GsView),
                                          c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "gs_plan_stage_times": (ctypes.c_int, [c_void_p, ctypes.POINTER(c_double),
                                           ctypes.POINTER(c_int64), c_int32]),
    "gs_last_error": (ctypes.c_char_p, []),
    "gs_probe_alu": (ctypes.c_int, [ctypes.POINTER(c_double), ctypes.POINTER(c_double), c_void_p]),
    "gs_server_create": (ctypes.c_int, [ctypes.POINTER(GsServerConfig), ctypes.POINTER(c_void_p)]),
    "gs_server_destroy": (None, [c_void_p]),
    "gs_server_add_model": (ctypes.c_int, [c_void_p, ctypes.POINTER(GsGaussians),
                                           ctypes.POINTER(c_int32)]),
    "gs_server_reserved_bytes": (ctypes.c_int, [c_void_p, ctypes.POINTER(c_int64)]),
    "gs_server_run": (ctypes.c_int, [c_void_p, ctypes.POINTER(GsRequest), c_int64, c_double,
                                     ctypes.POINTER(GsRequestResult), ctypes.POINTER(c_double)]),
    # gs_train.h
    "gs_project_bwd_stats": (ctypes.c_int, [ctypes.POINTER(GsGaussians), ctypes.POINTER(GsView),
                                            c_int32, c_float, c_void_p, ctypes.POINTER(GsGrads),
                                            c_int32, ctypes.POINTER(GsGradStats), c_void_p,
                                            c_void_p]),
    "gs_random_normals": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint64, c_int64, c_void_p,
                                         c_void_p]),
    "gs_adam_step": (ctypes.c_int, [ctypes.POINTER(GsParams), c_int64, ctypes.POINTER(GsGrads),
                                    ctypes.POINTER(GsAdamConfig), c_void_p]),
    "gs_params_activate": (ctypes.c_int, [ctypes.POINTER(GsParams), c_int64, c_void_p]),
    "gs_params_from_activated": (ctypes.c_int, [ctypes.POINTER(GsParams), c_int64, c_void_p]),
    "gs_densify": (ctypes.c_int, [ctypes.POINTER(GsParams), c_int64, ctypes.POINTER(GsGradStats),
                                  c_void_p, ctypes.POINTER(GsDensifyConfig),
                                  ctypes.POINTER(GsParams), c_int64, c_void_p,
                                  ctypes.POINTER(c_int64), c_void_p, c_void_p]),
    "gs_volume_metrics": (ctypes.c_int, [c_void_p, c_void_p, c_int32, c_int32, c_int32,
                                         ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                                         c_void_p, c_void_p]),
    "gs_train_config_default": (None, [ctypes.POINTER(GsTrainConfig)]),
    "gs_trainer_create": (ctypes.c_int, [ctypes.POINTER(GsTrainConfig), ctypes.POINTER(GsGaussians),
                                         c_void_p, ctypes.POINTER(GsView), c_int32,
                                         ctypes.POINTER(GsGrid), ctypes.POINTER(c_void_p)]),
    "gs_trainer_destroy": (None, [c_void_p]),
    "gs_trainer_run": (ctypes.c_int, [c_void_p, c_int32, c_void_p]),
    "gs_trainer_step": (ctypes.c_int, [c_void_p, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                                       c_void_p, ctypes.POINTER(c_float)]),
    "gs_trainer_model": (ctypes.c_int, [c_void_p, ctypes.POINTER(GsGaussians),
                                        ctypes.POINTER(c_int32)]),
    "gs_trainer_export": (ctypes.c_int, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                         ctypes.POINTER(c_int64)]),
    "gs_trainer_state": (ctypes.c_int, [c_void_p, ctypes.POINTER(GsParams), ctypes.POINTER(c_int64),
                                        ctypes.POINTER(GsGradStats)]),
    "gs_trainer_evaluate": (ctypes.c_int, [c_void_p, ctypes.POINTER(GsGrid), c_void_p, c_void_p,
                                           ctypes.POINTER(c_double), ctypes.POINTER(c_double)]),
}


def lib():
    """The loaded HIP library.  There is no fallback: a missing library is an
    error (build it with ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def call(name, *args):
    st = getattr(lib(), name)(*args)
    if st != 0:
        raise GsError(name, st, lib().gs_last_error().decode(errors="replace"))
