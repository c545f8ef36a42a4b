"""ctypes binding of libpt.so (include/pt.h): argument marshalling only.

Every step of the path runs in the HIP kernels of libpt.so; this module only
declares the C ABI.  It raises ImportError when the library has not been
built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PT_LIB names another build of the same sources (the host-sanitizer build of the CPU tests)
LIB_PATH = os.environ.get("PT_LIB") or os.path.join(HERE, "libpt.so")

PT_OK, PT_EINVAL, PT_ENOMEM, PT_EDEVICE, PT_EUNSUPPORTED, PT_EBUSY = 0, -1, -2, -3, -4, -5
MODES = {"incoherent": 0, "sorted": 1, "reuse": 2, "sorted_origin": 3, "sorted_reis": 4, "sorted_aila": 5,
         "reuse_plain": 6, "reuse_world": 7}
TIMER_KINDS = {0: "trace", 1: "raygen", 2: "shade", 3: "key", 4: "sort", 6: "other", 7: "shadow_trace",
               8: "shadow_accumulate"}


class PtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libpt error {status}: {msg}")
        self.status = status


class Material(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("albedo", C.c_float * 3), ("alpha", C.c_float),
                ("emission", C.c_float * 3)]


class Camera(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("look_at", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float)]


class Group(C.Structure):
    _fields_ = [("tile_w", C.c_uint16), ("tile_h", C.c_uint16), ("k", C.c_uint16),
                ("reuse_max_bounce", C.c_uint16), ("refill", C.c_uint16), ("waves_per_cu", C.c_uint16),
                ("leaf_gate", C.c_uint16), ("nee", C.c_uint16), ("traversal", C.c_uint16),
                ("frame_groups", C.c_uint16)]


class SceneDesc(C.Structure):
    _fields_ = [("tris", C.c_void_p), ("ntri", C.c_uint32), ("tri_mat", C.c_void_p),
                ("mats", C.c_void_p), ("nmat", C.c_uint32), ("env_radiance", C.c_float * 3)]


class SceneInfo(C.Structure):
    _fields_ = [("ntri", C.c_uint32), ("nnodes", C.c_uint32), ("max_depth", C.c_uint32),
                ("max_leaf", C.c_uint32), ("lo", C.c_float * 3), ("hi", C.c_float * 3),
                ("sah_cost", C.c_double), ("device_bytes", C.c_uint64), ("nemit", C.c_uint32),
                ("nnodes4", C.c_uint32), ("max_depth4", C.c_uint32), ("wide", C.c_uint32),
                ("quant", C.c_uint32)]


class Outputs(C.Structure):
    _fields_ = [("radiance", C.c_void_p), ("hit_prim", C.c_void_p), ("hit_t", C.c_void_p),
                ("ray_count", C.c_void_p), ("stats", C.c_void_p), ("rays", C.c_void_p), ("timer", C.c_void_p),
                ("shadow_count", C.c_void_p), ("touched", C.c_void_p), ("debug", C.c_void_p)]


class Job(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("camera", Camera), ("w", C.c_int32), ("h", C.c_int32),
                ("spp", C.c_int32), ("bounces", C.c_int32), ("mode", C.c_int32), ("reserved", C.c_int32),
                ("seed", C.c_uint64), ("radiance", C.c_void_p), ("hit_prim", C.c_void_p), ("hit_t", C.c_void_p)]


# name -> (restype, argtypes); the full list of exported entry points
_vp, _sz, _u32, _i32, _st = C.c_void_p, C.c_size_t, C.c_uint32, C.c_int, C.c_int32
PROTOTYPES = {
    "pt_probe_memory": (_st, [_vp, _sz, C.c_int32, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_float), _vp]),
    "pt_scene_create": (_st, [C.POINTER(SceneDesc), C.POINTER(_vp)]),
    "pt_scene_device_bytes": (_sz, [_vp]),
    "pt_scene_upload": (_st, [_vp, _vp, _sz, _vp]),
    "pt_scene_get_info": (_st, [_vp, C.POINTER(SceneInfo)]),
    "pt_scene_export_bvh": (_st, [_vp, _vp, _vp]),
    "pt_scene_export_bvh4": (_st, [_vp, _vp]),
    "pt_scene_export_bvh4q": (_st, [_vp, _vp]),
    "pt_scene_free": (_st, [_vp]),
    "pt_render_workspace_bytes": (_sz, [_i32, _i32, _i32, _i32, _i32, Group]),
    "pt_render": (_st, [_vp, C.POINTER(Camera), _i32, _i32, _i32, _i32, _i32, Group, C.c_uint64, _vp, _sz,
                        C.POINTER(Outputs), _vp]),
    "pt_trace_workspace_bytes": (_sz, []),
    "pt_trace": (_st, [_vp, _vp, _u32, _i32, _vp, _vp, _vp, _sz, _vp]),
    "pt_trace_static_scratch_bytes": (_sz, []),
    "pt_trace_static": (_st, [_vp, _vp, _u32, _i32, _i32, _vp, _vp, _vp]),
    "pt_ray_keys": (_st, [_vp, _vp, _u32, C.c_int, _vp, _vp]),
    "pt_sort_workspace_bytes": (_sz, [_u32]),
    "pt_sort_pairs": (_st, [_vp, _vp, _u32, _vp, _sz, _vp]),
    "pt_timer_create": (_st, [_i32, C.POINTER(_vp)]),
    "pt_timer_reset": (_st, [_vp]),
    "pt_timer_read": (_st, [_vp, _vp, _vp, _vp, _i32, C.POINTER(_i32)]),
    "pt_timer_free": (_st, [_vp]),
    "pt_device_info": (_st, [C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32)]),
    "pt_batch_job_bytes": (_sz, [C.POINTER(Job), Group]),
    "pt_batch_base_bytes": (_sz, [_i32]),
    "pt_batch_create": (_st, [_i32, Group, _vp, _sz, C.POINTER(_vp)]),
    "pt_batch_submit": (_st, [_vp, C.POINTER(Job), C.POINTER(_u32)]),
    "pt_batch_step": (_st, [_vp, _vp, C.POINTER(_i32)]),
    "pt_batch_poll": (_st, [_vp, _u32, C.POINTER(_i32)]),
    "pt_batch_release": (_st, [_vp, _u32]),
    "pt_batch_run": (_st, [_vp, _i32, _vp, _vp]),
    "pt_batch_free": (_st, [_vp]),
    "pt_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """Load libpt.so (built in-tree by paper_2310_07182_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2310_07182_amd.build.build() "
                              "(the HIP library is required, there is no fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != PT_OK:
        msg = lib().pt_last_error()
        raise PtError(status, msg.decode() if msg else "")
    return status
