"""ctypes declarations of the msim C-ABI (include/msim.h).  Argument
marshalling only: every step of the synthesis runs in libmsim.so."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsim.so")

MSIM_OK = 0
STATUS_NAMES = {
    0: "MSIM_OK", 1: "MSIM_E_INVALID_ARG", 2: "MSIM_E_OUTSIDE_ROOM", 3: "MSIM_E_TOO_CLOSE",
    4: "MSIM_E_SUPERSONIC", 5: "MSIM_E_WORKSPACE", 6: "MSIM_E_UNSUPPORTED", 7: "MSIM_E_HIP",
    8: "MSIM_E_DEVICE",
}


class MsimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


class Traj(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_points", C.c_int32), ("t", C.POINTER(C.c_double)),
                ("p", C.POINTER(C.c_double)), ("center", C.c_double * 3), ("radius", C.c_double),
                ("speed", C.c_double), ("phase0", C.c_double)]


class Scene(C.Structure):
    _fields_ = [("size", C.c_double * 3), ("beta", C.c_double * 6), ("src", Traj), ("rcv", Traj),
                ("n_mics", C.c_int32), ("mic_offset", C.POINTER(C.c_double)), ("max_order", C.c_int32),
                ("n_in", C.c_int64), ("n_out", C.c_int64)]


class Params(C.Structure):
    _fields_ = [("c", C.c_double), ("fs", C.c_double), ("taps", C.c_int32), ("kaiser_beta", C.c_double),
                ("cutoff", C.c_double), ("table_phases", C.c_int32), ("n_tiers", C.c_int32),
                ("tier_max_order", C.c_int32 * 4), ("tier_decim", C.c_int32 * 4), ("delay_model", C.c_int32),
                ("fd_kind", C.c_int32), ("farrow_order", C.c_int32), ("knot_slack", C.c_double),
                ("tier_mode", C.c_int32), ("tier_tol", C.c_double), ("tier_rmax", C.c_int32),
                ("adjx_mode", C.c_int32)]


class Profile(C.Structure):
    _fields_ = [("synth_ms", C.c_double), ("reduce_ms", C.c_double), ("adjx_ms", C.c_double),
                ("adjp_ms", C.c_double), ("params_ms", C.c_double), ("graph_ms", C.c_double),
                ("filter_ms", C.c_double),
                ("synth_launches", C.c_int32), ("reduce_launches", C.c_int32), ("adjx_launches", C.c_int32),
                ("adjp_launches", C.c_int32), ("params_launches", C.c_int32), ("graph_launches", C.c_int32),
                ("filter_launches", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("threads", C.c_int32), ("group_cap", C.c_int32), ("outputs_per_lane", C.c_int32),
                ("workgroups", C.c_int32), ("ms", C.c_double), ("adjx_gather", C.c_int32)]


class FdError(C.Structure):
    _fields_ = [("table", C.c_double), ("pair", C.c_double), ("farrow", C.c_double), ("budget", C.c_double),
                ("table_phases", C.c_int32)]


# name -> (argtypes); every function returns msim_status (int) except msim_last_error
_PLAN = C.c_void_p
SIGNATURES = {
    "msim_default_params": [C.POINTER(Params)],
    "msim_count_images": [C.c_int32, C.POINTER(C.c_int64)],
    "msim_suggest_n_out": [C.POINTER(Scene), C.POINTER(Params), C.POINTER(C.c_int64)],
    "msim_plan_create": [C.POINTER(Scene), C.c_int32, C.POINTER(Params), C.POINTER(_PLAN)],
    "msim_plan_destroy": [_PLAN],
    "msim_plan_layout": [_PLAN, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                         C.POINTER(C.c_int64)],
    "msim_plan_stats": [_PLAN, C.POINTER(C.c_int64), C.POINTER(C.c_double)],
    "msim_workspace_size": [_PLAN, C.c_int32, C.POINTER(C.c_size_t)],
    "msim_forward": [_PLAN, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p],
    "msim_forward_noalloc": [_PLAN, C.c_void_p, C.c_void_p, C.c_void_p],
    "msim_device_status": [_PLAN, C.c_void_p, C.POINTER(C.c_int32)],
    "msim_backward": [_PLAN, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                      C.c_size_t, C.c_void_p],
    "msim_backward_batched": [_PLAN, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_size_t, C.c_void_p, C.c_int32],
    "msim_plan_grad_layout": [_PLAN, C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
    "msim_batched_workspace_size": [_PLAN, C.POINTER(C.c_size_t)],
    "msim_forward_batched": [_PLAN, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_int32],
    "msim_get_tuning": [_PLAN, C.POINTER(Tuning)],
    "msim_get_fd_error": [_PLAN, C.POINTER(FdError)],
    "msim_plan_update": [_PLAN, C.c_void_p, C.c_void_p, C.c_void_p],
    "msim_get_images": [_PLAN, C.c_int32, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)],
    "msim_set_tuning": [_PLAN, C.POINTER(Tuning)],
    "msim_autotune_workspace_size": [_PLAN, C.POINTER(C.c_size_t)],
    "msim_autotune": [_PLAN, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_char_p,
                      C.POINTER(Tuning)],
    "msim_profile_begin": [_PLAN],
    "msim_profile_end": [_PLAN, C.POINTER(Profile)],
}

_lib = None


def load() -> C.CDLL:
    """Loads libmsim.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmsim.so is not built: run `python -m paper_2508_03065_amd.build` "
                              "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.msim_last_error.argtypes = []
        L.msim_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != MSIM_OK:
        raise MsimError(status, load().msim_last_error().decode(errors="replace"))
