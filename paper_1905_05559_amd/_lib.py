"""ctypes declarations of the C ABI in include/hess.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhess.so")

HESS_OK = 0
STATUS_NAMES = {
    0: "HESS_OK", 1: "HESS_E_ARG", 2: "HESS_E_SHAPE", 3: "HESS_E_LABEL", 4: "HESS_E_NONFINITE",
    5: "HESS_E_WORKSPACE", 6: "HESS_E_BUDGET", 7: "HESS_E_DEVICE", 8: "HESS_E_NOCONV",
    9: "HESS_E_NOTPD", 10: "HESS_E_UNSUPPORTED",
}
ACT = {"tanh": 0, "sigmoid": 1, "relu": 2}
DTYPE = {"float64": 0, "float32": 1}
PREC = {"f64": 0, "f32": 1, "bf16": 2, "f32_split": 3}
OP = {"exact": 0, "opg": 1, "hvp": 2, "topk": 3, "predvar": 4, "batched": 5, "exact_cols": 6, "curvature": 7, "syev": 8}
OPT = {"check_inputs": 0, "hbm_budget": 1, "fault_after": 2, "profile": 3, "graphs": 4, "autotune": 5,
       "factor_bytes": 6}

# Every symbol include/hess.h declares.
EXPORTS = (
    "hess_create", "hess_destroy", "hess_status_str", "hess_last_error", "hess_set_option", "hess_autotune_report",
    "hess_num_params", "hess_workspace_size", "hess_exact", "hess_opg", "hess_hvp", "hess_exact_cols",
    "hess_topk_eig", "hess_predvar", "hess_profile_read", "hess_profile_reset", "hess_batched",
    "hess_server_create", "hess_server_submit", "hess_server_wait", "hess_server_stats", "hess_server_destroy",
    "hess_mfma_stream_rate", "hess_hvp_prepare", "hess_hvp_apply", "hess_hvp_release", "hess_curvature",
    "hess_syev", "hess_curvature_noalloc",
)


class HessMlp(C.Structure):
    _fields_ = [("L", C.c_int32), ("T", C.POINTER(C.c_int64)), ("act", C.POINTER(C.c_int32)),
                ("dtype", C.c_int32), ("W", C.POINTER(C.c_void_p)), ("b", C.POINTER(C.c_void_p))]


class HessData(C.Structure):
    _fields_ = [("N", C.c_int64), ("dtype", C.c_int32), ("X", C.c_void_p), ("Y", C.c_void_p)]


class HessEigOpts(C.Structure):
    _fields_ = [("which", C.c_int32), ("source", C.c_int32), ("M", C.c_void_p), ("M_dtype", C.c_int32),
                ("prec", C.c_int32), ("P", C.c_int64), ("oversample", C.c_int64),
                ("max_iter", C.c_int32), ("tol", C.c_double), ("seed", C.c_uint64), ("method", C.c_int32),
                ("block", C.c_int32)]


class HessEigInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("applies", C.c_int32), ("max_rel_residual", C.c_double),
                ("shift_used", C.c_double)]


class HessRequest(C.Structure):
    _fields_ = [("kind", C.c_int32), ("model", HessMlp), ("data", HessData), ("H", C.c_void_p), ("G", C.c_void_p),
                ("K", C.c_int64), ("lam", C.c_void_p), ("Q", C.c_void_p), ("tol", C.c_double), ("seed", C.c_uint64),
                ("delta", C.c_double), ("nq", C.c_int64), ("Xq", C.c_void_p), ("cls", C.c_void_p), ("s", C.c_void_p),
                ("curv_mode", C.c_int32), ("lam_tilde", C.c_double), ("fault_launch", C.c_int32)]


class HessProfEntry(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("ms", C.c_double), ("flops", C.c_double),
                ("bytes", C.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libhess.so; raises ImportError (never falls back) when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libhess.so not found at %s: build it with "
                          "`python -m paper_1905_05559_amd.build`" % path)
    lib = C.CDLL(path)
    vp, i32, i64, st = C.c_void_p, C.c_int32, C.c_int64, C.c_int
    pm, pd = C.POINTER(HessMlp), C.POINTER(HessData)
    sig = {
        "hess_create": (st, [C.POINTER(vp), C.c_int, vp]),
        "hess_destroy": (st, [vp]),
        "hess_status_str": (C.c_char_p, [st]),
        "hess_last_error": (C.c_char_p, [vp]),
        "hess_set_option": (st, [vp, C.c_int, i64]),
        "hess_num_params": (st, [pm, C.POINTER(i64)]),
        "hess_workspace_size": (st, [vp, C.c_int, pm, pd, C.c_int, i64, vp, C.POINTER(C.c_size_t)]),
        "hess_exact": (st, [vp, pm, pd, C.c_int, vp, vp, C.c_size_t]),
        "hess_opg": (st, [vp, pm, pd, C.c_int, vp, vp, C.c_size_t]),
        "hess_hvp": (st, [vp, pm, pd, C.c_int, i64, vp, vp, vp, C.c_size_t]),
        "hess_exact_cols": (st, [vp, pm, pd, C.c_int, i64, i64, vp, vp, C.c_size_t]),
        "hess_autotune_report": (st, [vp, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]),
        "hess_mfma_stream_rate": (st, [vp, C.c_int, i64, vp, C.POINTER(C.c_double)]),
        "hess_hvp_prepare": (st, [vp, pm, pd, C.c_int, i64, vp, C.c_size_t, C.POINTER(vp)]),
        "hess_hvp_apply": (st, [vp, vp, i64, vp, vp]),
        "hess_hvp_release": (st, [vp]),
        "hess_curvature": (st, [vp, C.c_int, i64, i64, vp, vp, C.c_double, i64, vp, vp, vp, C.c_size_t]),
        "hess_curvature_noalloc": (st, [vp, C.c_int, i64, i64, vp, vp, C.c_double, i64, vp, vp]),
        "hess_syev": (st, [vp, i64, vp, i64, vp, vp, vp, C.c_size_t]),
        "hess_topk_eig": (st, [vp, pm, pd, i64, C.POINTER(HessEigOpts), vp, vp,
                               C.POINTER(HessEigInfo), vp, C.c_size_t]),
        "hess_predvar": (st, [vp, pm, i64, vp, vp, C.c_double, i64, vp, vp, vp, vp, C.c_size_t]),
        "hess_profile_read": (C.c_int, [vp, C.POINTER(HessProfEntry), C.c_int]),
        "hess_profile_reset": (st, [vp]),
        "hess_batched": (st, [vp, i64, pm, pd, C.c_int, C.POINTER(vp), C.POINTER(vp), vp, C.c_size_t]),
        "hess_server_create": (st, [C.POINTER(vp), C.c_int, C.c_int, vp, C.c_size_t, C.c_int]),
        "hess_server_submit": (st, [vp, C.POINTER(HessRequest), C.POINTER(C.c_uint64)]),
        "hess_server_wait": (st, [vp, C.c_uint64, C.POINTER(C.c_double)]),
        "hess_server_stats": (st, [vp, C.POINTER(C.c_int64)]),
        "hess_server_destroy": (st, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
