"""ctypes declarations of libgicp.so (the C ABI in include/gicp.h)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgicp.so")

GICP_OK, GICP_E_ARG, GICP_E_NONFINITE, GICP_E_NO_CORR, GICP_E_DEGENERATE, GICP_E_OOM, GICP_E_HIP, \
    GICP_E_INEXACT, GICP_E_TOO_LARGE = range(9)
NOALLOC_MAX_POINTS = 131072
REG_NONE, REG_PLANE, REG_ELLIPSE = 0, 1, 2
ACC_TWOSUM, ACC_FP32, ACC_FP64 = 0, 1, 2


class Params(C.Structure):
    _fields_ = [
        ("k", C.c_int32),
        ("eps", C.c_float),
        ("r_max", C.c_float),
        ("max_it", C.c_int32),
        ("conv_rot", C.c_double),
        ("conv_trans", C.c_double),
        ("reg_mode", C.c_int32),
        ("cell_src", C.c_float),
        ("precision", C.c_int32),
        ("flags", C.c_int32),
        ("lanes", C.c_int32),
    ]


FLAG_MULTI_LAUNCH = 1
FLAG_QUEUE = 2
FLAG_GRAPH = 4
FLAG_NO_REUSE = 8


class Problem(C.Structure):
    _fields_ = [
        ("src", C.c_void_p),
        ("src_covs", C.c_void_p),
        ("n", C.c_int64),
        ("map", C.c_void_p),
        ("init_pose", C.c_double * 16),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("iters", C.c_int32),
        ("n_inliers", C.c_int32),
        ("cost", C.c_double),
        ("converged", C.c_int32),
        ("status", C.c_int32),
        ("hip_error", C.c_int32),
        ("reserved", C.c_int32),
    ]


class Frame(C.Structure):
    _fields_ = [
        ("src", C.c_void_p),
        ("src_covs", C.c_void_p),
        ("n", C.c_int64),
    ]


MOTION_PREVIOUS, MOTION_CONSTANT_VELOCITY = 0, 1


class MlpPair(C.Structure):
    _fields_ = [
        ("src", C.c_void_p),
        ("n_src", C.c_int64),
        ("tgt", C.c_void_p),
        ("n_tgt", C.c_int64),
        ("src_idx", C.c_void_p),
        ("tgt_idx", C.c_void_p),
    ]


MLP_POINTS, MLP_PARAMS, MLP_BF16, MLP_CACHE, MLP_SCALE, MLP_MAX_BATCH = 4096, 75462, 40960, 640, 0.5, 4096

P = C.c_void_p
I64 = C.c_int64
D16 = C.c_double * 16
D36 = C.c_double * 36
D6 = C.c_double * 6

SIGNATURES = {
    "gicp_params_default": (None, [C.POINTER(Params)]),
    "gicp_version": (C.c_char_p, []),
    "gicp_strerror": (C.c_char_p, [C.c_int]),
    "gicp_create": (C.c_int, [C.POINTER(P), C.c_int]),
    "gicp_destroy": (C.c_int, [P]),
    "gicp_sync_status": (C.c_int, [P, P]),
    "gicp_estimate_cell": (C.c_int, [P, P, I64, C.c_int, C.POINTER(C.c_float), P]),
    "gicp_knn": (C.c_int, [P, P, I64, P, I64, C.c_int, C.c_float, C.c_float, P, P, P]),
    "gicp_covariances": (C.c_int, [P, P, I64, C.c_int, C.c_float, C.c_int, C.c_float, P, P]),
    "gicp_covariances_noalloc": (C.c_int, [P, P, I64, C.c_int, C.c_float, C.c_int, C.c_float, P, P]),
    "gicp_map_build": (C.c_int, [P, P, P, I64, C.c_float, C.c_int, C.c_float, C.POINTER(P), P]),
    "gicp_map_destroy": (C.c_int, [P]),
    "gicp_map_info": (C.c_int, [P, C.POINTER(I64), C.POINTER(C.c_float)]),
    "gicp_map_nearest": (C.c_int, [P, P, P, I64, C.c_float, P, P, P, P, C.c_int32, P]),
    "gicp_register": (C.c_int, [P, P, P, I64, P, D16, C.POINTER(Params), D16, D36, D6, P,
                                C.POINTER(Stats), P]),
    "gicp_register_dev": (C.c_int, [P, P, P, I64, P, P, C.POINTER(Params), P, P, P, P, P, P]),
    "gicp_track": (C.c_int, [P, C.c_int, C.POINTER(Frame), P, D16, C.c_int, C.POINTER(Params), P, P, P,
                             C.POINTER(Stats), P]),
    "gicp_register_pair": (C.c_int, [P, P, P, I64, P, P, I64, C.c_float, D16, C.POINTER(Params), D16, D36,
                                     D6, C.POINTER(Stats), P]),
    "gicp_register_batch": (C.c_int, [P, C.c_int, C.POINTER(Problem), C.POINTER(Params), P, P, P,
                                      C.POINTER(Stats), P]),
    "gicp_profile": (C.c_int, [P, C.c_int]),
    "gicp_profile_read": (C.c_int, [P, C.c_int, C.POINTER(I64), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "gicp_depth_to_points": (C.c_int, [P, P, C.c_int, C.c_int, C.c_float, C.c_float, C.c_float, C.c_float,
                                       C.c_float, C.c_float, P, I64, C.POINTER(I64), P]),
    "gicp_keyframe_gaussians": (C.c_int, [P, P, P, I64, P, D16, C.c_float, C.c_float, P, P, C.POINTER(I64),
                                          C.POINTER(C.c_double), P]),
    "gicp_keyframe_policy": (C.c_int, [C.c_double, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int]),
    "gicp_map_insert": (C.c_int, [P, P, P, P, I64, P]),
    "gicp_mlp_init": (C.c_int, [P, C.c_uint64, P, P, P, P, P]),
    "gicp_mlp_sync_weights": (C.c_int, [P, P, P, P]),
    "gicp_mlp_pack": (C.c_int, [P, C.c_int, C.POINTER(MlpPair), P, P, P]),
    "gicp_mlp_forward": (C.c_int, [P, C.c_int, P, P, P, P, P, P, P, P]),
    "gicp_mlp_backward": (C.c_int, [P, C.c_int, P, P, P, P, P, P, P, P]),
    "gicp_mlp_adam_step": (C.c_int, [P, P, P, P, P, C.c_int, C.c_float, P, P]),
}

PROF_LINEARIZE, PROF_KNN_COV, PROF_GRID, PROF_SOLVE = 0, 1, 2, 3
KEYFRAME, MAPPING_ONLY = 1, 2

_lib = None


def load(path: str = ""):
    """Loads libgicp.so (built in-tree by ``build.py``; $GICP_LIBRARY names
    another build of the same library).  Raises if it is missing: there is
    no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("GICP_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"libgicp.so not built ({path}); run paper_2403_12550_amd/build.py")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
