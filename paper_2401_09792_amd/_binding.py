"""ctypes declarations of the libgtucker C ABI (include/gtucker.h).  Marshalling only."""

from __future__ import annotations

import ctypes as C
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libgtucker.so")
_lib = None

GT_OK = 0
STATUS_NAMES = {0: "GT_OK", 1: "GT_ERR_ARG", 2: "GT_ERR_SHAPE", 3: "GT_ERR_RANK",
                4: "GT_ERR_WORKSPACE", 5: "GT_ERR_UNSUPPORTED", 6: "GT_ERR_HIP",
                7: "GT_ERR_NO_DEVICE"}
GT_FIT_WARM_START = 1
GT_C64, GT_C128 = 0, 1
GT_INTERF_NONE, GT_INTERF_PAPER, GT_INTERF_ALL = 0, 1, 2
DEV_NONFINITE, DEV_EIG_SWEEPS, DEV_CHOLESKY, DEV_ZERO_STREAM = 1, 2, 4, 8


class ChannelDesc(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nt", C.c_int32), ("nsc", C.c_int32),
                ("group_size", C.c_int32), ("m", C.c_int32), ("n", C.c_int32),
                ("p", C.c_int32), ("ns", C.c_int32), ("a_id", C.c_int32),
                ("b_id", C.c_int32), ("serving", C.c_int32)]


class Offsets(C.Structure):
    _fields_ = [("x", C.c_int64), ("a", C.c_int64), ("b", C.c_int64), ("c", C.c_int64),
                ("g", C.c_int64), ("ht", C.c_int64), ("sc", C.c_int64),
                ("n_groups", C.c_int32), ("reserved", C.c_int32)]


class FitOptions(C.Structure):
    _fields_ = [("iters", C.c_int32), ("ttm_prec", C.c_int32), ("eig_fp64", C.c_int32),
                ("flags", C.c_uint32), ("dtype", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("bstep", C.c_int32), ("tpass", C.c_int32), ("split", C.c_int32),
                ("probe_ms", C.c_float)]


# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "gt_plan_create": (C.c_int, [C.POINTER(ChannelDesc), C.c_int32, C.POINTER(FitOptions),
                                 C.POINTER(C.c_void_p)]),
    "gt_plan_destroy": (None, [C.c_void_p]),
    "gt_plan_offsets": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Offsets)]),
    "gt_plan_totals": (C.c_int, [C.c_void_p, C.POINTER(Offsets), C.POINTER(C.c_int32)]),
    "gt_plan_workspace_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "gt_workspace_init": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "gt_tucker_fit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                C.c_void_p]),
    "gt_tucker_reconstruct": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_size_t, C.c_void_p]),
    "gt_sinr_eval": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_float),
                               C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                               C.c_void_p]),
    "gt_sinr_eval_system": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_float),
                                      C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_size_t, C.c_void_p]),
    "gt_sinr_eval_full": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_float), C.c_int32,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                    C.c_void_p]),
    "gt_combine_full": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                  C.c_void_p, C.c_size_t, C.c_void_p]),
    "gt_combine_compressed": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t,
                                        C.c_void_p]),
    "gt_sinr_eval_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.POINTER(C.c_float), C.c_int32, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_size_t, C.c_void_p]),
    "gt_sinr_eval_backward_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p,
                                               C.POINTER(C.c_float), C.c_int32, C.c_void_p,
                                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gt_tucker_reconstruct_backward": (C.c_int, [C.c_void_p] * 11 + [C.c_void_p, C.c_size_t,
                                                                      C.c_void_p]),
    "gt_tucker_fit_backward": (C.c_int, [C.c_void_p]),
    "gt_plan_autotune": (C.c_int, [C.c_void_p] * 7 + [C.c_size_t, C.c_void_p,
                                                       C.POINTER(TuneResult)]),
    "gt_plan_set_tuning": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]),
    "gt_status_string": (C.c_char_p, [C.c_int]),
    "gt_last_error_detail": (C.c_char_p, []),
    "gt_profile_enable": (C.c_int, [C.c_int32]),
    "gt_profile_reset": (C.c_int, []),
    "gt_profile_query": (C.c_int, [C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
}


def lib_path() -> str:
    return _LIB_PATH


def load() -> C.CDLL:
    """Loads the in-tree shared library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"libgtucker.so not built ({_LIB_PATH}); run __graft_entry__.build()")
    lib = C.CDLL(_LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class GtError(RuntimeError):
    def __init__(self, where: str, code: int):
        lib = load()
        detail = lib.gt_last_error_detail().decode()
        msg = f"{where}: {STATUS_NAMES.get(code, code)} ({lib.gt_status_string(code).decode()})"
        if detail and code == 6:
            msg += f": {detail}"
        super().__init__(msg)
        self.code = code


def check(where: str, code: int) -> None:
    if code != GT_OK:
        raise GtError(where, code)
