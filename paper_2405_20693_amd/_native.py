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
    "gs_loss_tv": (ctypes.c_int, [c_void_p, c_int32, c_int32, c_int32, c_float, c_void_p, c_void_p,
                                  c_int32, c_void_p, c_void_p]),
    "gs_plan_set_timing": (ctypes.c_int, [c_void_p, c_int32]),
    "gs_plan_stage_times": (ctypes.c_int, [c_void_p, ctypes.POINTER(c_double),
                                           ctypes.POINTER(c_int64), c_int32]),
    "gs_last_error": (ctypes.c_char_p, []),
    "gs_server_create": (ctypes.c_int, [ctypes.POINTER(GsServerConfig), ctypes.POINTER(c_void_p)]),
    "gs_server_destroy": (None, [c_void_p]),
    "gs_server_add_model": (ctypes.c_int, [c_void_p, ctypes.POINTER(GsGaussians),
                                           ctypes.POINTER(c_int32)]),
    "gs_server_run": (ctypes.c_int, [c_void_p, ctypes.POINTER(GsRequest), c_int64, c_double,
                                     ctypes.POINTER(GsRequestResult), ctypes.POINTER(c_double)]),
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
