"""ctypes declarations of the libdpmt C ABI (include/dpmt.h)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int16, c_int32, c_int64, c_void_p, c_char_p

# DPMT_LIBRARY names another build of the library (the sanitizer build of the
# host runtime that the CPU tests load); the default is the in-tree build.
LIB_PATH = os.environ.get("DPMT_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdpmt.so")

DPMT_OK = 0
DPMT_E_INVALID = -1
DPMT_E_STATE = -2
DPMT_E_RANK = -3
DPMT_E_NOMEM = -4
DPMT_E_DEVICE = -5
DPMT_E_UNSUPPORTED = -6

DT_NOALLOC_MAX_SIDE = 16384        # DPMT_DT_NOALLOC_MAX_SIDE
DT_NOALLOC_MAX_CELLS = 2097152     # DPMT_DT_NOALLOC_MAX_CELLS
HOG_MAX_SIDE = 65536               # DPMT_HOG_MAX_SIDE
DT_WINDOW = 0                      # DPMT_DT_WINDOW
DT_ENVELOPE = 1                    # DPMT_DT_ENVELOPE
DT_METHODS = {"window": DT_WINDOW, "envelope": DT_ENVELOPE}

DIRECT_FP32 = 0
TENSOR_FP32 = 1
TENSOR_BF16 = 2
TENSOR_FP8 = 3
CP_FP32 = 4

MODES = {"direct_fp32": DIRECT_FP32, "tensor_fp32": TENSOR_FP32,
         "tensor_bf16": TENSOR_BF16, "tensor_fp8": TENSOR_FP8, "cp_fp32": CP_FP32}

LAUNCH_BATCHED = 0
LAUNCH_PER_LEVEL = 1
LAUNCH_GRAPH = 2
LAUNCH_OVERLAP = 3
LAUNCHES = {"batched": LAUNCH_BATCHED, "per_level": LAUNCH_PER_LEVEL, "graph": LAUNCH_GRAPH,
            "overlap": LAUNCH_OVERLAP}


class Shape(ctypes.Structure):
    _fields_ = [("h", c_int32), ("w", c_int32)]


class Component(ctypes.Structure):
    _fields_ = [("root", c_int32), ("n_parts", c_int32), ("parts", POINTER(c_int32)),
                ("anchors", POINTER(c_int32)), ("deform", POINTER(c_float))]


class LevelDesc(ctypes.Structure):
    _fields_ = [("cell_offset", c_int64), ("rows", c_int32), ("cols", c_int32)]


class PyramidDesc(ctypes.Structure):
    _fields_ = [("n_levels", c_int32), ("levels", POINTER(LevelDesc)), ("octave", c_int32)]


class HogLevel(ctypes.Structure):
    _fields_ = [("cell_offset", c_int64), ("rows", c_int32), ("cols", c_int32),
                ("pad_rows", c_int32), ("pad_cols", c_int32), ("cell", c_int32),
                ("inv_scale", c_float)]


class Hypothesis(ctypes.Structure):
    _fields_ = [("image", c_int32), ("level", c_int32), ("comp", c_int32), ("y", c_int32), ("x", c_int32)]


class Layout(ctypes.Structure):
    _fields_ = [("n_score", c_int64), ("n_offsets", c_int64), ("n_maps", c_int32),
                ("map_image", POINTER(c_int32)), ("map_level", POINTER(c_int32)),
                ("map_comp", POINTER(c_int32)), ("map_rows", POINTER(c_int32)),
                ("map_cols", POINTER(c_int32)), ("map_score_off", POINTER(c_int64)),
                ("map_offs_off", POINTER(c_int64)), ("n_cells", c_int64), ("n_resp", c_int64),
                ("n_resp_root", c_int64), ("n_resp_part", c_int64),
                ("workspace_bytes", c_int64)]


# name -> (restype, argtypes); every symbol include/dpmt.h declares
SIGNATURES = {
    "dpmt_create": (c_int32, [POINTER(c_void_p), c_int32, c_void_p]),
    "dpmt_destroy": (None, [c_void_p]),
    "dpmt_load_filters": (c_int32, [c_void_p, c_int32, POINTER(Shape), POINTER(c_float), c_int32,
                                    POINTER(Component)]),
    "dpmt_decompose": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double)]),
    "dpmt_decompose_cp": (c_int32, [c_void_p, POINTER(c_int32), c_int32, c_double, POINTER(c_double)]),
    "dpmt_select_ranks": (c_int32, [c_void_p, c_double, c_int32, c_int32, POINTER(c_int32), POINTER(c_double)]),
    "dpmt_set_thresholds": (c_int32, [c_void_p, POINTER(c_float)]),
    "dpmt_fit_thresholds": (c_int32, [c_void_p, POINTER(c_float), c_int32, POINTER(Hypothesis), c_float,
                                      POINTER(c_float)]),
    "dpmt_load_cp": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_float)]),
    "dpmt_get_cp": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_float), POINTER(c_int64)]),
    "dpmt_plan": (c_int32, [c_void_p, c_int32, POINTER(PyramidDesc), POINTER(POINTER(Layout))]),
    "dpmt_score_pyramid": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "dpmt_level_responses": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_int32, c_void_p,
                                       c_int64, POINTER(c_int64), c_void_p]),
    "dpmt_distance_transform": (c_int32, [c_void_p, c_int32, c_int32, c_int32, POINTER(c_float),
                                          c_void_p, c_void_p, c_void_p, c_void_p]),
    "dpmt_distance_transform_noalloc": (c_int32, [c_void_p, c_int32, c_int32, c_int32, POINTER(c_float),
                                                  c_void_p, c_void_p, c_void_p, c_void_p]),
    "dpmt_distance_transform_method": (c_int32, [c_void_p, c_int32, c_int32, c_int32, POINTER(c_float),
                                                 c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "dpmt_set_profiling": (c_int32, [c_void_p, c_int32]),
    "dpmt_stage_times": (c_int32, [c_void_p, POINTER(c_float), c_int32, POINTER(c_int32)]),
    "dpmt_set_launch": (c_int32, [c_void_p, c_int32]),
    "dpmt_tile_config_count": (c_int32, []),
    "dpmt_tile_config_name": (c_char_p, [c_int32]),
    "dpmt_set_tile_config": (c_int32, [c_void_p, c_int32, c_int32]),
    "dpmt_get_tile_config": (c_int32, [c_void_p, c_int32]),
    "dpmt_autotune": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32,
                                POINTER(c_float), POINTER(c_int32), c_void_p]),
    "dpmt_detect": (c_int32, [c_void_p, c_void_p, c_float, c_void_p, c_int64, c_void_p, c_void_p]),
    "dpmt_hog_pyramid": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_int32, POINTER(HogLevel),
                                   c_void_p, c_void_p]),
    "dpmt_status_string": (c_char_p, [c_int32]),
    "dpmt_last_error": (c_char_p, [c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libdpmt.so (built in-tree by ``python -m paper_1707_03268_amd.build``).

    Raises ImportError when the library has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libdpmt.so not found at {path}; build it with "
                          "`python -m paper_1707_03268_amd.build` (or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
