"""ctypes declarations of the C ABI in include/xpcs.h (libxpcs.so, built in-tree).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libxpcs.so")

XPCS_OK = 0
XPCS_EINVAL = -1
XPCS_ENOMEM = -2
XPCS_ERANGE = -3
XPCS_EBUDGET = -4
XPCS_EDEVICE = -5
XPCS_EUNSUPPORTED = -6
XPCS_EQUEUED = -7
STATUS_NAMES = {0: "XPCS_OK", -1: "XPCS_EINVAL", -2: "XPCS_ENOMEM", -3: "XPCS_ERANGE",
                -4: "XPCS_EBUDGET", -5: "XPCS_EDEVICE", -6: "XPCS_EUNSUPPORTED", -7: "XPCS_EQUEUED"}

XPCS_STREAM_QUEUED = 1
XPCS_STREAM_ADMITTED = 2
XPCS_STREAM_FAILED = 3

XPCS_U8 = 1
XPCS_U16 = 2
XPCS_F32 = 10
XPCS_F64 = 11
XPCS_PREC_BF16 = 0
XPCS_PREC_FP8 = 1
XPCS_BASIS_RANDOMIZED = 0
XPCS_BASIS_EXACT = 1
XPCS_ALL_ROIS = -1


class XpcsFactors(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int64), ("N", ctypes.c_int64),
        ("k", ctypes.c_int32), ("n_roi", ctypes.c_int32),
        ("U", ctypes.c_void_p), ("sigma", ctypes.c_void_p), ("V", ctypes.c_void_p),
        ("roi_npix", ctypes.c_void_p), ("roi_sum", ctypes.c_void_p), ("roi_gram", ctypes.c_void_p),
    ]


class XpcsCompressOpts(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32), ("oversample", ctypes.c_int32),
        ("power_iters", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("basis", ctypes.c_void_p),
        ("method", ctypes.c_int32), ("reserved", ctypes.c_int32), ("spectrum", ctypes.c_void_p),
    ]


class XpcsStreamDesc(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int64), ("dtype", ctypes.c_int32), ("n_roi", ctypes.c_int32),
        ("k", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("roi_label", ctypes.c_void_p), ("basis", ctypes.c_void_p),
        ("window", ctypes.c_int64), ("max_block", ctypes.c_int64),
    ]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_ST = ctypes.c_int32

SIGNATURES = {
    "xpcs_create": (_ST, [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_P)]),
    "xpcs_destroy": (None, [_P]),
    "xpcs_set_stream": (_ST, [_P, _P]),
    "xpcs_sync": (_ST, [_P]),
    "xpcs_last_error": (ctypes.c_char_p, [_P]),
    "xpcs_workspace_bytes": (ctypes.c_size_t, [_P]),
    "compress_frames": (_ST, [_P, _P, _I32, _I64, _I64, _P, _I32,
                              ctypes.POINTER(XpcsCompressOpts), ctypes.POINTER(XpcsFactors)]),
    "correlate_two_time": (_ST, [_P, ctypes.POINTER(XpcsFactors), _I32, _I64, _I64, _P, _I32, _I64,
                                 _P, _P]),
    "correlate_two_time_noalloc": (_ST, [_P, ctypes.POINTER(XpcsFactors), _I32, _I64, _I64, _P, _I32, _I64,
                                         _P, _P]),
    "correlate_two_time_raw": (_ST, [_P, _P, _I32, _I64, _I64, _P, _I32, _I32, _I64, _I64, _P, _I32,
                                     _I64, _P, _P, _P]),
    "g2_from_two_time": (_ST, [_P, _P, _I32, _I64, _I64, _P, _P]),
    "g2_from_factors": (_ST, [_P, ctypes.POINTER(XpcsFactors), _I32, _I64, _I64, _P, _P]),
    "fit_relaxation": (_ST, [_P, _P, _P, _I64, _I32, _I64, _I64, _P, _I32, _P, _P]),
    "two_time_stats": (_ST, [_P, ctypes.POINTER(XpcsFactors), _I32, _I64, _I64, _P, _P, _P]),
    "fit_relaxation_stretched": (_ST, [_P, _P, _P, _I64, _I32, _I64, _I64, _P, _I32, _P, _P]),
    "xpcs_rank_rule": (_ST, [_P, _P, _I64, ctypes.c_double, _P]),
    "peak_visibility": (_ST, [_P, _P, _P, _I32, _I64, _I64, _I64, _I64, _I64, _P, ctypes.c_double, _P, _P]),
    "shifted_texture_frames": (_ST, [_P, _P, _I32, _I64, _I64, _I64, ctypes.c_uint64, _P]),
    "xpcs_factors_save": (_ST, [_P, ctypes.POINTER(XpcsFactors), _P, ctypes.c_uint64, ctypes.c_char_p]),
    "xpcs_factors_info": (_ST, [ctypes.c_char_p, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I32),
                                ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_uint64)]),
    "xpcs_factors_load": (_ST, [_P, ctypes.c_char_p, ctypes.POINTER(XpcsFactors), _P]),
    "xpcs_stream_save": (_ST, [_P, ctypes.c_char_p]),
    "xpcs_stream_load": (_ST, [_P, ctypes.c_char_p, ctypes.POINTER(_P)]),
    "xpcs_enable_phase_timing": (_ST, [_P, _I32]),
    "xpcs_phase_filter": (_ST, [_P, ctypes.c_char_p]),
    "xpcs_phase_times": (_ST, [_P, _I32, _P, _P, _P, ctypes.POINTER(_I32)]),
    "xpcs_stream_open": (_ST, [_P, ctypes.POINTER(XpcsStreamDesc), ctypes.POINTER(_P)]),
    "xpcs_stream_push": (_ST, [_P, _P, _I64, _P, _I32]),
    "xpcs_stream_g2": (_ST, [_P, _P, _P]),
    "xpcs_stream_frames": (_I64, [_P]),
    "xpcs_stream_close": (None, [_P]),
    "xpcs_server_create": (_ST, [ctypes.c_int, ctypes.c_size_t, _I32, _I32, ctypes.POINTER(_P)]),
    "xpcs_server_destroy": (None, [_P]),
    "xpcs_server_last_error": (ctypes.c_char_p, [_P]),
    "xpcs_server_open": (_ST, [_P, ctypes.POINTER(XpcsStreamDesc), ctypes.POINTER(_I64), ctypes.POINTER(_I32)]),
    "xpcs_server_state": (_ST, [_P, _I64, ctypes.POINTER(_I32)]),
    "xpcs_server_push": (_ST, [_P, _I64, _P, _I64, _P, _I32, _P]),
    "xpcs_server_poll": (_ST, [_P, _I64, _I32, _P, _P, ctypes.POINTER(_I32)]),
    "xpcs_server_g2": (_ST, [_P, _I64, _P, _P]),
    "xpcs_server_wait": (_ST, [_P, _I64]),
    "xpcs_server_close": (_ST, [_P, _I64]),
    "xpcs_server_stats": (_ST, [_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libxpcs.so once; raise ImportError if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python -m paper_2407_20356_amd.build` "
            "(the library has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
