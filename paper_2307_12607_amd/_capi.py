"""ctypes declarations of libexwarp's C-ABI (include/exwarp.h).

Loading fails loudly when the library has not been built: there is no other
implementation of the warp in this package.
"""

from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libexwarp.so")

EXW_F32, EXW_F16, EXW_BF16 = 0, 1, 2
EXW_SUCCESS, EXW_ERROR_INVALID_VALUE, EXW_ERROR_UNSUPPORTED, EXW_ERROR_LAUNCH = 0, 1, 2, 3
EXW_ABI_VERSION = 2
EXW_MAX_PHASES = 4
EXW_MAX_CHANNELS = 64
EXW_NO_ALLOC_SCRATCH_BYTES = 1 << 20
EXW_EMD_MAX_BINS = 4096

# name -> (restype, argtypes), in the order of include/exwarp.h
_i32 = ctypes.c_int32
_p = ctypes.c_void_p
_sz = ctypes.c_size_t
_f = ctypes.c_float
SIGNATURES = {
    "exw_abi_version": (ctypes.c_int, []),
    "exw_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "exw_last_error": (ctypes.c_char_p, []),
    "exw_warp_forward_batched": (ctypes.c_int, [_p, ctypes.c_int, _i32, _i32, _i32, _i32, _p, _p,
                                                _i32, _p, _p, _p, _p]),
    "exw_warp_forward": (ctypes.c_int, [_p, ctypes.c_int, _i32, _i32, _i32, _p, _f, _p, _p, _p]),
    "exw_warp_backward_workspace_bytes": (_sz, [ctypes.c_int, _i32, _i32, _i32, _i32]),
    "exw_warp_backward_batched": (ctypes.c_int, [_p, ctypes.c_int, _i32, _i32, _i32, _i32, _p, _p,
                                                 _i32, _p, _p, _p, _p, _sz, _p]),
    "exw_warp_backward": (ctypes.c_int, [_p, ctypes.c_int, _i32, _i32, _i32, _p, _f, _p, _p, _p,
                                         _p, _sz, _p]),
    "exw_warp_forward_batched_record": (ctypes.c_int, [_p, ctypes.c_int, _i32, _i32, _i32, _i32,
                                                       _p, _p, _i32, _p, _p, _p, _p, _p, _sz,
                                                       _p]),
    "exw_warp_backward_batched_recorded": (ctypes.c_int, [_p, ctypes.c_int, _i32, _i32, _i32, _i32,
                                                          _p, _p, _i32, _p, _p, _p, _p, _sz, _p]),
    "exw_motion_stats_workspace_bytes": (_sz, [_i32, _i32, _i32]),
    "exw_motion_stats": (ctypes.c_int, [_p, _i32, _i32, _i32, _p, _p, _sz, _p]),
    "exw_motion_stats_no_alloc": (ctypes.c_int, [_p, _i32, _i32, _i32, _p, _p]),
    "exw_frame_quality_workspace_bytes": (_sz, [_i32, _i32, _i32, _i32]),
    "exw_decision_plan": (ctypes.c_int, [_i32, _i32, _i32, _p]),
    "exw_threshold_policy": (ctypes.c_int, [_p, _p, ctypes.c_double, ctypes.c_double, _p]),
    "exw_warp_chain": (ctypes.c_int, [_p, ctypes.c_int, _i32, _i32, _i32, _i32, _p, _f, _i32, _p,
                                      _p, _p, _p]),
    "exw_frame_quality": (ctypes.c_int, [_p, _p, ctypes.c_int, _i32, _i32, _i32, _i32,
                                         ctypes.c_double, _p, _p, _sz, _p]),
    "exw_buffer_emd_workspace_bytes": (_sz, [_i32, _i32, _i32]),
    "exw_buffer_emd": (ctypes.c_int, [_p, _p, ctypes.c_int, _i32, _i32, _i32, _i32,
                                      ctypes.c_double, ctypes.c_double, _i32, _p, _p, _sz, _p]),
    "exw_dynamic_objects_workspace_bytes": (_sz, [_i32, _i32, _i32]),
    "exw_dynamic_objects": (ctypes.c_int, [_p, _i32, _i32, _i32, _i32, _p, _p, _sz, _p]),
    "exw_stream_copy": (ctypes.c_int, [_p, _p, _sz, _p]),
    "exw_stream_read": (ctypes.c_int, [_p, _sz, _p, _p]),
    "exw_stream_write": (ctypes.c_int, [_p, _sz, _p]),
}


EXW_DECIDE_NONE, EXW_DECIDE_WARP, EXW_DECIDE_EXTRAPOLATE = -1, 0, 1
EXW_SHOW_REPEAT, EXW_SHOW_WARP, EXW_SHOW_EXTRAPOLATE = 0, 1, 2
EXW_FROM_RENDERED, EXW_FROM_P1, EXW_FROM_P2 = 0, 1, 2


class DisplayPlan(ctypes.Structure):
    """exw_display_plan of include/exwarp.h."""
    _fields_ = [("scenario", ctypes.c_int32), ("kind", ctypes.c_int32 * 3),
                ("source", ctypes.c_int32 * 3), ("node", ctypes.c_int32 * 3),
                ("new_frames", ctypes.c_int32)]


class ExwError(RuntimeError):
    """A libexwarp call returned a status other than EXW_SUCCESS."""

    def __init__(self, status: int, name: str, detail: str):
        self.status = status
        super().__init__(f"{name}: {status_string(status)}: {detail}")


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"libexwarp.so not found at {LIB_PATH}; build it first with "
                "`python -m paper_2307_12607_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.exw_abi_version() != EXW_ABI_VERSION:
            raise ImportError(f"libexwarp ABI {L.exw_abi_version()} != {EXW_ABI_VERSION}")
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().exw_status_string(int(status)).decode()


def last_error() -> str:
    return lib().exw_last_error().decode()


def check(status: int, name: str) -> None:
    if status != EXW_SUCCESS:
        raise ExwError(status, name, last_error())
