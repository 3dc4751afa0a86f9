"""ctypes mirror of include/dr.h and loader of the in-tree libdr.so.

There is no fallback: if the HIP library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdr.so")

MAX_TEX = 3
MAX_VIEWS = 16
BG_ID = 0xFFFFFFFF
NOALLOC_SCRATCH_BYTES = 128 << 20      # DR_NOALLOC_SCRATCH_BYTES

PROBE_CONTIGUOUS, PROBE_LINES, PROBE_SCATTERED, PROBE_CONFLICTING = 0, 1, 2, 3
PROBE_SQRT, PROBE_RCP = 0, 1

STATUS = {0: "ok", -1: "invalid argument", -2: "out of device memory", -3: "HIP error", -4: "unsupported"}


class Scene(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tris", C.c_int32),
                ("tri", C.c_void_p), ("corner_uv", C.c_void_p),
                ("n_tex", C.c_int32),
                ("tex_w", C.c_int32 * MAX_TEX), ("tex_h", C.c_int32 * MAX_TEX),
                ("tex_c", C.c_int32 * MAX_TEX),
                ("shading", C.c_int32), ("tex_mode", C.c_int32),
                ("light_dir", C.c_float * 3), ("light_rgb", C.c_float * 3),
                ("ambient", C.c_float), ("diffuse", C.c_float), ("layers", C.c_int32),
                ("n_ctrl", C.c_int32), ("sub_rowptr", C.c_void_p), ("sub_cols", C.c_void_p),
                ("sub_w", C.c_void_p)]


class View(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("view_proj", C.c_float * 16),
                ("cam_pos", C.c_float * 3), ("near_w", C.c_float)]


class Tuning(C.Structure):
    _fields_ = [("tile_px", C.c_int32), ("bin_capacity", C.c_int32), ("items_per_launch", C.c_int32)]


class Perturb(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("step", C.c_uint32), ("pair", C.c_uint32),
                ("scene_index", C.c_uint32), ("sign", C.c_int32), ("eps", C.c_float * (1 + MAX_TEX))]


class Optim(C.Structure):
    _fields_ = [("kind", C.c_int32), ("averaging", C.c_int32), ("lr", C.c_float * (1 + MAX_TEX)),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps_hat", C.c_float)]


class Stats(C.Structure):
    _fields_ = [("tile_overflows", C.c_uint64), ("saturations", C.c_uint64), ("nonfinite", C.c_uint64),
                ("max_bin", C.c_uint64), ("full_scans", C.c_uint64)]


class BatchScene(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("views", C.POINTER(View)), ("n_views", C.c_int32),
                ("targets", C.c_void_p), ("theta", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p),
                ("Q", C.c_void_p), ("K", C.c_void_p), ("eps", C.c_float * (1 + MAX_TEX)),
                ("lr", C.c_float * (1 + MAX_TEX)), ("bin_capacity", C.c_int32)]


class Timing(C.Structure):
    _fields_ = [("signs_ms", C.c_double), ("setup_ms", C.c_double), ("tile_ms", C.c_double),
                ("fold_ms", C.c_double), ("step_ms", C.c_double),
                ("signs_launches", C.c_int64), ("setup_launches", C.c_int64), ("tile_launches", C.c_int64),
                ("fold_launches", C.c_int64), ("step_launches", C.c_int64)]


# exported entry points: name -> (restype, argtypes)
_vp = C.c_void_p
SIGNATURES = {
    "dr_create": (C.c_int, [C.POINTER(_vp), C.POINTER(Scene), C.POINTER(Tuning), _vp]),
    "dr_destroy": (C.c_int, [_vp]),
    "dr_set_stream": (C.c_int, [_vp, _vp]),
    "dr_set_tuning": (C.c_int, [_vp, C.POINTER(Tuning)]),
    "dr_set_scene_index": (C.c_int, [_vp, C.c_uint32]),
    "dr_param_count": (C.c_int64, [_vp]),
    "dr_group_count": (C.c_int64, [_vp]),
    "dr_render": (C.c_int, [_vp, _vp, C.POINTER(View), C.POINTER(Perturb), _vp, _vp, _vp]),
    "dr_loss": (C.c_int, [_vp, _vp, C.POINTER(View), C.c_int32, _vp, _vp]),
    "dr_signs": (C.c_int, [_vp, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _vp]),
    "dr_estimate_grad": (C.c_int, [_vp, _vp, C.POINTER(View), C.c_int32, _vp, C.c_uint64, C.c_uint32,
                                   C.c_int32, C.POINTER(C.c_float), _vp, _vp]),
    "dr_estimate_grad_full": (C.c_int, [_vp, _vp, C.POINTER(View), C.c_int32, _vp, C.c_uint64, C.c_uint32,
                                        C.c_int32, C.POINTER(C.c_float), _vp, _vp]),
    "dr_estimate_grad_image": (C.c_int, [_vp, _vp, C.POINTER(View), C.c_int32, _vp, C.c_uint64, C.c_uint32,
                                         C.c_int32, C.POINTER(C.c_float), _vp, _vp]),
    "dr_estimate_grad_noalloc": (C.c_int, [_vp, _vp, C.POINTER(View), C.c_int32, _vp, C.c_uint64, C.c_uint32,
                                           C.c_int32, C.POINTER(C.c_float), _vp, _vp]),
    "dr_subdivide_sizes": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "dr_subdivide": (C.c_int, [_vp, _vp, C.c_int32, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp]),
    "dr_set_adaptive_bins": (C.c_int, [_vp, C.c_int32]),
    "dr_get_tuning": (C.c_int, [_vp, C.POINTER(Tuning)]),
    "dr_decode_grad": (C.c_int, [_vp, _vp, _vp, C.POINTER(C.c_float), C.c_int32, C.c_int32, _vp]),
    "dr_step": (C.c_int, [_vp, _vp, _vp, _vp, C.c_uint32, _vp, _vp, C.POINTER(C.c_float), C.c_int32,
                          C.POINTER(Optim)]),
    "dr_timing_enable": (C.c_int, [_vp, C.c_int]),
    "dr_timing_read": (C.c_int, [_vp, C.POINTER(Timing), C.c_int]),
    "dr_stats": (C.c_int, [_vp, C.POINTER(Stats)]),
    "dr_reset_stats": (C.c_int, [_vp]),
    "dr_batch_create": (C.c_int, [C.POINTER(_vp), C.POINTER(BatchScene), C.c_int32, C.c_int32, C.c_int32,
                                  C.POINTER(Optim), C.c_uint64, C.c_uint32, _vp]),
    "dr_batch_destroy": (C.c_int, [_vp]),
    "dr_batch_estimate": (C.c_int, [_vp]),
    "dr_batch_step": (C.c_int, [_vp, C.c_int]),
    "dr_batch_set_step": (C.c_int, [_vp, C.c_uint32]),
    "dr_batch_get_step": (C.c_int, [_vp, C.POINTER(C.c_uint32)]),
    "dr_batch_stats": (C.c_int, [_vp, C.POINTER(Stats)]),
    "dr_batch_timing_enable": (C.c_int, [_vp, C.c_int]),
    "dr_batch_timing_read": (C.c_int, [_vp, C.POINTER(Timing), C.c_int]),
    "dr_batch_last_error": (C.c_char_p, [_vp]),
    "dr_probe_atomics": (C.c_int, [_vp, C.c_int64, C.c_int32, C.c_int32, C.c_int64, _vp]),
    "dr_probe_math": (C.c_int, [C.c_int32, C.c_uint32, C.c_uint32, _vp, _vp, _vp]),
    "dr_status_str": (C.c_char_p, [C.c_int]),
    "dr_last_error": (C.c_char_p, [_vp]),
}

_lib = None


def load():
    """Load libdr.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
