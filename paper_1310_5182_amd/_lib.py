"""ctypes loader of liblagp_alc.so (the gfx950 library).  No fallback: if the
library is missing or fails to load, every call raises."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblagp_alc.so")

LAGP_OK = 0
LAGP_EINVAL = -1
LAGP_EWORKSPACE = -2
LAGP_EHIP = -3
LAGP_EUNSUPPORTED = -4

LAGP_FP64 = 0
LAGP_MIXED = 1
LAGP_FP64_REFORM = 2

LAGP_ABI_VERSION = 3
LAGP_NORMALIZE_ALC = 1
LAGP_NN_BRUTE = 2
LAGP_PLAN_NO_TUNE = 1
LAGP_PLAN_SCHEDULES = 6


class Problem(ctypes.Structure):
    """lagp_problem of include/lagp_alc.h (same field order and types)."""

    _fields_ = [("struct_size", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("X", ctypes.c_void_p), ("Y", ctypes.c_void_p), ("XX", ctypes.c_void_p),
                ("N", ctypes.c_int64), ("M", ctypes.c_int64),
                ("p", ctypes.c_int32), ("n0", ctypes.c_int32), ("n", ctypes.c_int32), ("Np", ctypes.c_int32),
                ("n_per", ctypes.c_void_p), ("Np_per", ctypes.c_void_p), ("d_per", ctypes.c_void_p),
                ("d", ctypes.c_double), ("g", ctypes.c_double),
                ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("d_sep", ctypes.c_void_p)]


class Outputs(ctypes.Structure):
    """lagp_outputs of include/lagp_alc.h (same field order and types)."""

    _fields_ = [("struct_size", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("mean", ctypes.c_void_p), ("s2", ctypes.c_void_p), ("var", ctypes.c_void_p),
                ("sel", ctypes.c_void_p), ("sel_off", ctypes.c_void_p),
                ("alc", ctypes.c_void_p), ("alc32", ctypes.c_void_p), ("pool", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("guard", ctypes.c_void_p)]

# Every symbol declared in include/lagp_alc.h.
EXPORTS = (
    "lagp_nn_pool",
    "lagp_nn_pool_workspace",
    "lagp_nn_pool_ws",
    "lagp_nn_pool_static",
    "lagp_nn_pool_grouped",
    "lagp_alc_scores",
    "lagp_mspe_workspace",
    "lagp_mspe_from_pool",
    "lagp_alc_from_pool",
    "lagp_alc_workspace",
    "lagp_alc_predict",
    "lagp_abi_version",
    "lagp_alc_uneven_workspace",
    "lagp_alc_uneven_from_pool",
    "lagp_plan_create",
    "lagp_plan_launch",
    "lagp_plan_describe",
    "lagp_plan_destroy",
    "lagp_local_nll",
    "lagp_local_nll_backward",
    "lagp_local_mle_d",
    "lagp_local_predict",
    "lagp_status_string",
    "lagp_last_error",
    "lagp_version",
)

_lib = None


class LagpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(msg)
        self.code = code


def load():
    """Load the library (once).  Raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} not found: build it with `python -m paper_1310_5182_amd.build` "
            "(or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    P, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.lagp_nn_pool.argtypes = [P, i64, i32, P, i64, i32, P, P]
    L.lagp_nn_pool.restype = i32
    L.lagp_nn_pool_workspace.argtypes = [i64, i32, i64, ctypes.POINTER(ctypes.c_size_t)]
    L.lagp_nn_pool_workspace.restype = i32
    L.lagp_nn_pool_ws.argtypes = [P, i64, i32, P, i64, i32, P, P, ctypes.c_size_t, P]
    L.lagp_nn_pool_ws.restype = i32
    L.lagp_nn_pool_static.argtypes = [P, i64, i32, P, i64, i32, P, P]
    L.lagp_nn_pool_static.restype = i32
    L.lagp_nn_pool_grouped.argtypes = [P, i64, i32, P, i64, i32, i32, P, P, ctypes.c_size_t, P]
    L.lagp_nn_pool_grouped.restype = i32
    L.lagp_mspe_workspace.argtypes = [i64, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
    L.lagp_mspe_workspace.restype = i32
    L.lagp_mspe_from_pool.argtypes = [P, P, i64, i32, P, i64, P, i32, i32, i32, f64, f64, P, P, P, P, P, P, P,
                                      ctypes.c_size_t, P]
    L.lagp_mspe_from_pool.restype = i32
    L.lagp_alc_scores.argtypes = [P, i32, i32, P, P, i64, P, P, f64, f64, i32, P, P]
    L.lagp_alc_scores.restype = i32
    L.lagp_alc_from_pool.argtypes = [P, P, i64, i32, P, i64, P, i32, i32, i32, f64, f64, i32,
                                     P, P, P, P, P, P, P, P, P]
    L.lagp_alc_from_pool.restype = i32
    PP, PO = ctypes.POINTER(Problem), ctypes.POINTER(Outputs)
    L.lagp_alc_workspace.argtypes = [PP, ctypes.POINTER(ctypes.c_size_t)]
    L.lagp_alc_workspace.restype = i32
    L.lagp_alc_predict.argtypes = [PP, PO, P, ctypes.c_size_t, P]
    L.lagp_alc_predict.restype = i32
    L.lagp_abi_version.argtypes = []
    L.lagp_abi_version.restype = i32
    L.lagp_alc_uneven_workspace.argtypes = [i32, i64, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
    L.lagp_alc_uneven_workspace.restype = i32
    L.lagp_alc_uneven_from_pool.argtypes = [P, P, i64, i32, P, i64, P, i32, i32, i32, P, P, P, P, f64, f64,
                                            i32, P, P, P, P, P, P, P, P, ctypes.c_size_t, P]
    L.lagp_alc_uneven_from_pool.restype = i32
    L.lagp_plan_create.argtypes = [PP, PO, P, ctypes.c_size_t, i32, P, ctypes.POINTER(ctypes.c_void_p)]
    L.lagp_plan_create.restype = i32
    L.lagp_plan_launch.argtypes = [P, P]
    L.lagp_plan_launch.restype = i32
    L.lagp_plan_describe.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t]
    L.lagp_plan_describe.restype = i32
    L.lagp_plan_destroy.argtypes = [P]
    L.lagp_plan_destroy.restype = i32
    L.lagp_local_nll.argtypes = [P, P, i64, i32, P, i64, i32, P, P, P, P, P, P, P, P]
    L.lagp_local_nll.restype = i32
    L.lagp_local_nll_backward.argtypes = [P, P, i64, i32, P, i64, i32, P, P, P, P, P, P]
    L.lagp_local_nll_backward.restype = i32
    L.lagp_local_mle_d.argtypes = [P, P, i64, i32, P, i64, i32, P, f64, f64, f64, i32, P, P, P, P, P]
    L.lagp_local_mle_d.restype = i32
    L.lagp_local_predict.argtypes = [P, P, i64, i32, P, i64, i32, P, P, f64, P, P, P, P, P]
    L.lagp_local_predict.restype = i32
    L.lagp_status_string.argtypes = [i32]
    L.lagp_status_string.restype = ctypes.c_char_p
    L.lagp_last_error.argtypes = []
    L.lagp_last_error.restype = ctypes.c_char_p
    L.lagp_version.argtypes = []
    L.lagp_version.restype = ctypes.c_char_p
    _lib = L
    return L


def check(code: int) -> None:
    if code == LAGP_OK:
        return
    L = load()
    msg = f"{L.lagp_status_string(code).decode()}: {L.lagp_last_error().decode()}"
    if code == LAGP_EINVAL:
        raise ValueError(msg)
    raise LagpError(code, msg)
