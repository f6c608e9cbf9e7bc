"""ctypes declarations of the libsrt C ABI (mirrors include/srt.h)."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# SRT_LIB_PATH selects another build of the same library (e.g. a variant
# compiled with different flags); the default is the in-tree build.
LIB_PATH = os.environ.get("SRT_LIB_PATH") or os.path.join(_PKG, "libsrt.so")

SRT_NUM_COUNTERS = 8
NOALLOC_SCRATCH_BYTES = 64 << 20  # SRT_NOALLOC_SCRATCH_BYTES in include/srt.h
COUNTER_NAMES = ["traversals", "nodes", "prims", "candidates", "philox", "deep", "ray_samples",
                 "lost"]


class SrtScene(C.Structure):
    _fields_ = [("num_gaussians", C.c_int64), ("sh_degree", C.c_int32),
                ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p)]


class SrtBuildOpts(C.Structure):
    _fields_ = [("width", C.c_int32), ("leaf_size", C.c_int32), ("size_split", C.c_int32)]


class SrtBvhInfo(C.Structure):
    _fields_ = [("num_gaussians", C.c_int64), ("num_nodes", C.c_int64), ("width", C.c_int32),
                ("leaf_size", C.c_int32), ("depth", C.c_int32), ("sh_degree", C.c_int32),
                ("device_bytes", C.c_int64)]


class SrtRays(C.Structure):
    _fields_ = [("count", C.c_int64), ("origins", C.c_void_p), ("dirs", C.c_void_p),
                ("tmin", C.c_void_p), ("tmax", C.c_void_p), ("ignore_gid", C.c_void_p),
                ("ray_ids", C.c_void_p), ("sample_ids", C.c_void_p), ("purpose", C.c_uint32)]


class SrtTraceOpts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("spp", C.c_int32), ("n_per_traversal", C.c_int32),
                ("sample_offset", C.c_uint32), ("bg", C.c_float * 3), ("any_hit", C.c_int32),
                ("stack_limit", C.c_int32), ("depth_mode", C.c_int32),
                ("depth_axis", C.c_float * 3), ("image_width", C.c_int32),
                ("persistent", C.c_int32), ("refill_threshold", C.c_int32),
                ("estimator", C.c_int32), ("rng", C.c_int32),
                ("walk", C.c_int32)]


class SrtCamera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("forward", C.c_float * 3), ("right", C.c_float * 3),
                ("up", C.c_float * 3), ("tan_half", C.c_float), ("width", C.c_int32),
                ("height", C.c_int32), ("jitter", C.c_float * 2)]


class SrtPathmixOpts(C.Structure):
    _fields_ = [("light", C.c_float * 3), ("plane_y", C.c_float), ("tmin_secondary", C.c_float),
                ("stages", C.c_int32)]


class SrtBatch(C.Structure):
    _fields_ = [("num_views", C.c_int32), ("cameras", C.c_void_p), ("spp", C.c_void_p),
                ("extra", SrtRays), ("extra_spp", C.c_int32), ("ray_id_base", C.c_uint32)]


class SrtTuning(C.Structure):
    _fields_ = [("persistent", C.c_int32), ("refill_threshold", C.c_int32),
                ("waves_per_cu", C.c_int32), ("lds_stack", C.c_int32)]


# name -> (restype, argtypes)
PROTOTYPES = {
    "srt_status_str": (C.c_char_p, [C.c_int]),
    "srt_version": (C.c_int32, []),
    "srt_build_bvh": (C.c_int, [C.POINTER(SrtScene), C.POINTER(SrtBuildOpts), C.c_void_p,
                                C.POINTER(C.c_void_p)]),
    "srt_destroy_bvh": (None, [C.c_void_p]),
    "srt_set_memory_limit": (C.c_int, [C.c_int64]),
    "srt_memory_stats": (C.c_int, [C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "srt_refit_bvh": (C.c_int, [C.c_void_p, C.POINTER(SrtScene), C.c_void_p]),
    "srt_bvh_get_info": (C.c_int, [C.c_void_p, C.POINTER(SrtBvhInfo)]),
    "srt_bvh_records": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p]),
    "srt_bvh_nodes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "srt_trace_workspace_size": (C.c_size_t, [C.c_void_p, C.c_int64]),
    "srt_trace_forward": (C.c_int, [C.c_void_p, C.POINTER(SrtRays), C.POINTER(SrtTraceOpts),
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_size_t, C.c_void_p]),
    "srt_trace_forward_noalloc": (C.c_int, [C.c_void_p, C.POINTER(SrtRays),
                                            C.POINTER(SrtTraceOpts), C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_void_p, C.c_void_p]),
    "srt_backward_workspace_size": (C.c_size_t, [C.c_void_p, C.c_int64]),
    "srt_trace_backward": (C.c_int, [C.c_void_p, C.POINTER(SrtScene), C.POINTER(SrtRays),
                                     C.POINTER(SrtTraceOpts), C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                     C.c_void_p]),
    "srt_camera_rays": (C.c_int, [C.POINTER(SrtCamera), C.c_void_p, C.c_void_p, C.c_void_p]),
    "srt_pathmix_workspace_size": (C.c_size_t, [C.c_void_p, C.POINTER(SrtCamera), C.c_int32]),
    "srt_trace_pathmix": (C.c_int, [C.c_void_p, C.POINTER(SrtCamera), C.c_uint32,
                                    C.POINTER(SrtTraceOpts), C.POINTER(SrtPathmixOpts),
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "srt_batch_plan_create": (C.c_int, [C.c_void_p, C.POINTER(SrtBatch), C.POINTER(SrtTraceOpts),
                                        C.POINTER(SrtTuning), C.c_void_p,
                                        C.POINTER(C.c_void_p)]),
    "srt_batch_plan_destroy": (None, [C.c_void_p]),
    "srt_batch_plan_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]),
    "srt_batch_plan_execute": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p]),
    "srt_batch_plan_execute_eager": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                               C.c_void_p]),
}

_lib = None


class SrtError(RuntimeError):
    def __init__(self, fn, code):
        name = load().srt_status_str(code).decode() if _lib is not None else str(code)
        super().__init__(f"{fn} failed: {name} ({code})")
        self.code = code


def load():
    """Load libsrt.so; fails loudly when the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libsrt.so not found at {LIB_PATH}: build it with "
                              "`python -m paper_2504_06598_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(fn_name, code):
    if code != 0:
        raise SrtError(fn_name, code)
