"""ctypes mirror of include/salf.h and the loader of the in-tree libsalf.so.

Argument marshalling only: every step of rendering runs in the library's HIP kernels.  There
is no fallback: if the library is missing or fails to load, importing raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsalf.so")

SALF_OK = 0
STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "OUT_OF_MEMORY", -3: "DEVICE", -4: "NOT_FOUND", -5: "BUDGET",
                -6: "BUSY", -7: "UNSUPPORTED", -8: "TRUNCATED"}
FIELD_CORNER, FIELD_PAPER, FIELD_SDF = 0, 1, 2
SCENE_PREACTIVATE = 1
SCHEDULE_NONE, SCHEDULE_BUILD, SCHEDULE_REUSE = 0, 1, 2
MAX_INDEX_LEVEL = 6  # SALF_MAX_INDEX_LEVEL
ERR_OUT_OF_MEMORY = -2
PINHOLE, FISHEYE_EQUIDISTANT, LIDAR_SPINNING = 0, 1, 2


class SceneDesc(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("root_size", C.c_double), ("root_dims", C.c_int32 * 3),
                ("max_level", C.c_int32), ("field", C.c_int32), ("flags", C.c_int32)]


class RefineOpts(C.Structure):
    _fields_ = [("grad_threshold", C.c_double), ("alpha_min", C.c_double)]


class Actor(C.Structure):
    _fields_ = [("scene_id", C.c_int32), ("R", C.c_float * 9), ("t", C.c_float * 3)]


class SceneStats(C.Structure):
    _fields_ = [("n_voxels", C.c_int64), ("n_nodes", C.c_int64), ("n_root_cells", C.c_int64),
                ("n_occupied_roots", C.c_int64), ("workspace_bytes", C.c_size_t)]


class Sensor(C.Structure):
    _fields_ = [("model", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float), ("max_theta", C.c_float),
                ("elev_min", C.c_float), ("elev_max", C.c_float), ("az0", C.c_float), ("t0", C.c_float),
                ("dt_line", C.c_float), ("R0", C.c_float * 9), ("p0", C.c_float * 3), ("v", C.c_float * 3),
                ("w", C.c_float * 3), ("t_near", C.c_float), ("t_far", C.c_float)]


class Rays(C.Structure):
    _fields_ = [("o", C.c_void_p), ("d", C.c_void_p), ("n", C.c_int64), ("t_near", C.c_float),
                ("t_far", C.c_float), ("image_width", C.c_int32), ("reserved", C.c_int32)]


class RenderOpts(C.Structure):
    _fields_ = [("samples_per_voxel", C.c_int32), ("t_min", C.c_float), ("background", C.c_float * 3),
                ("schedule", C.c_int32), ("d_work", C.c_void_p), ("work_bytes", C.c_size_t),
                ("pieces", C.c_int32), ("reserved", C.c_int32)]


class Outputs(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("opacity", C.c_void_p), ("intensity", C.c_void_p),
                ("t_end", C.c_void_p), ("n_hits", C.c_void_p), ("hit_voxel", C.c_void_p), ("hit_t", C.c_void_p),
                ("hit_capacity", C.c_int32), ("reserved", C.c_int32)]


class RenderItem(C.Structure):
    _fields_ = [("scene_id", C.c_int32), ("reserved", C.c_int32), ("sensor", C.POINTER(Sensor)),
                ("opts", RenderOpts), ("out", Outputs)]


class GradsIn(C.Structure):
    _fields_ = [("d_rgb", C.c_void_p), ("d_depth", C.c_void_p), ("d_opacity", C.c_void_p),
                ("d_intensity", C.c_void_p)]


class ServerOpts(C.Structure):
    _fields_ = [("d_pool", C.c_void_p), ("pool_bytes", C.c_size_t), ("d_work", C.c_void_p),
                ("work_bytes", C.c_size_t), ("max_batch", C.c_int32), ("max_inflight", C.c_int32),
                ("max_launch_rays", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("released", C.c_int64),
                ("launches", C.c_int64), ("pool_in_use", C.c_size_t), ("pool_peak", C.c_size_t),
                ("queued", C.c_int32), ("inflight", C.c_int32)]


# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "salf_abi_version": (C.c_int32, []),
    "salf_last_error": (C.c_char_p, []),
    "salf_create": (C.c_int32, [C.c_int32, C.POINTER(C.c_void_p)]),
    "salf_destroy": (C.c_int32, [C.c_void_p]),
    "salf_sync": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "salf_scene_workspace_size": (C.c_int32, [C.POINTER(SceneDesc), C.c_int64, C.POINTER(C.c_size_t)]),
    "salf_scene_create": (C.c_int32, [C.c_void_p, C.POINTER(SceneDesc), C.c_int64, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
                                      C.POINTER(C.c_int32)]),
    "salf_scene_refresh": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "salf_refine_work_size": (C.c_int32, [C.c_int64, C.POINTER(C.c_size_t)]),
    "salf_refine": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(RefineOpts), C.c_void_p,
                                C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                C.POINTER(C.c_int64), C.c_void_p]),
    "salf_render_composite": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_void_p]),
    "salf_scene_index_size": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "salf_scene_build_index": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p]),
    "salf_scene_get_stats": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(SceneStats)]),
    "salf_scene_destroy": (C.c_int32, [C.c_void_p, C.c_int32]),
    "salf_sensor_ray_count": (C.c_int32, [C.POINTER(Sensor), C.POINTER(C.c_int64)]),
    "salf_generate_rays": (C.c_int32, [C.c_void_p, C.POINTER(Sensor), C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p]),
    "salf_render": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Sensor), C.POINTER(Rays), C.POINTER(RenderOpts),
                                C.POINTER(Outputs), C.c_void_p]),
    "salf_render_static": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Sensor), C.POINTER(Rays),
                                       C.POINTER(RenderOpts), C.POINTER(Outputs), C.c_void_p]),
    "salf_raster_work_size": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Sensor), C.c_int64,
                                          C.POINTER(C.c_size_t)]),
    "salf_render_raster": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Sensor), C.POINTER(RenderOpts),
                                       C.POINTER(Outputs), C.c_void_p, C.c_size_t, C.POINTER(C.c_int64), C.c_void_p]),
    "salf_render_multi_work_size": (C.c_int32, [C.c_int32, C.POINTER(C.c_size_t)]),
    "salf_render_multi": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "salf_render_work_size": (C.c_int32, [C.POINTER(Sensor), C.POINTER(Rays), C.POINTER(C.c_size_t)]),
    "salf_render_schedule": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Sensor), C.POINTER(Rays),
                                         C.POINTER(RenderOpts), C.c_void_p]),
    "salf_trace_hits": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Rays), C.c_int32, C.c_int32,
                                    C.POINTER(RenderOpts), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    "salf_set_step_budget": (C.c_int32, [C.c_void_p, C.c_int32]),
    "salf_render_backward": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Sensor), C.POINTER(Rays),
                                         C.POINTER(RenderOpts), C.POINTER(Outputs), C.POINTER(GradsIn), C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p]),
    "salf_server_work_size": (C.c_int32, [C.POINTER(ServerOpts), C.POINTER(C.c_size_t)]),
    "salf_server_request_bytes": (C.c_int32, [C.POINTER(Sensor), C.c_uint32, C.POINTER(C.c_size_t)]),
    "salf_server_create": (C.c_int32, [C.c_void_p, C.POINTER(ServerOpts), C.POINTER(C.c_void_p)]),
    "salf_server_submit": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Sensor), C.POINTER(RenderOpts), C.c_uint32,
                                       C.POINTER(C.c_uint64)]),
    "salf_server_poll": (C.c_int32, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(Outputs),
                                     C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "salf_server_wait": (C.c_int32, [C.c_void_p, C.c_uint64, C.c_double, C.POINTER(C.c_int32)]),
    "salf_server_release": (C.c_int32, [C.c_void_p, C.c_uint64]),
    "salf_server_get_stats": (C.c_int32, [C.c_void_p, C.POINTER(ServerStats)]),
    "salf_server_destroy": (C.c_int32, [C.c_void_p]),
}

_lib = None


class SalfError(RuntimeError):
    def __init__(self, status, func, msg):
        super().__init__(f"{func} failed with {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """The loaded libsalf.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python paper_2507_18713_amd/build.py`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def call(name, *args):
    """Call an entry point and raise SalfError on a non-zero status."""
    st = getattr(lib(), name)(*args)
    if st != SALF_OK:
        msg = lib().salf_last_error()
        raise SalfError(st, name, msg.decode() if msg else "")
    return st
