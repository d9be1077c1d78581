"""ctypes declarations for libdedisp.so (argument marshalling only; the C ABI is include/dedisp.h)."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdedisp.so")

DD_OK = 0
DD_FILLING = 1
DD_WARN_CAND_OVERFLOW = 2
DD_ERR_INVALID_ARG = -1
DD_ERR_TOO_SHORT = -2
DD_ERR_SEQUENCE = -3
DD_ERR_WORKSPACE = -4
DD_ERR_HIP = -5
DD_ERR_UNSUPPORTED = -6
DD_F32, DD_F16, DD_U8 = 0, 1, 2
DD_FORM_AUTO, DD_FORM_LDS, DD_FORM_REGWIN, DD_FORM_DIRECT = 0, 1, 2, 3
CHAN_BLOCK = 32


class Tuning(C.Structure):
    _fields_ = [("dms_per_wave", C.c_int32), ("waves", C.c_int32),
                ("samples_per_lane", C.c_int32), ("chan_stage", C.c_int32),
                ("producer_waves", C.c_int32), ("kernel_form", C.c_int32)]


class BinnedRun(C.Structure):
    _fields_ = [("log2", C.c_int32), ("d0", C.c_int32), ("d1", C.c_int32), ("maxdelay", C.c_int32),
                ("nout", C.c_int64), ("kernel_form", C.c_int32), ("dms_per_wave", C.c_int32), ("waves", C.c_int32),
                ("producer_waves", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("nchan", C.c_int32), ("ndm", C.c_int32), ("in_dtype", C.c_int32),
                ("maxdelay", C.c_int32), ("nsamp", C.c_int64), ("nout", C.c_int64),
                ("workspace_bytes", C.c_int64), ("ring_bytes", C.c_int64),
                ("dms_per_wave", C.c_int32), ("waves", C.c_int32),
                ("samples_per_lane", C.c_int32), ("max_span", C.c_int32),
                ("adds", C.c_int64), ("chan_stage", C.c_int32), ("producer_waves", C.c_int32),
                ("launch_copies", C.c_int32), ("launch_buf", C.c_int32), ("launch_stage", C.c_int32),
                ("launch_ring", C.c_int32), ("launch_lds", C.c_int64),
                ("kernel_form", C.c_int32), ("window_chunks", C.c_int32),
                ("stream_workspace_bytes", C.c_int64)]


class Cand(C.Structure):
    _fields_ = [("dm_index", C.c_int32), ("reserved", C.c_int32), ("t", C.c_int64),
                ("value", C.c_float), ("snr", C.c_float)]


class BatchItem(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("d_in", C.c_void_p), ("nsamp", C.c_int64),
                ("in_row_stride", C.c_int64), ("d_out", C.c_void_p), ("out_row_stride", C.c_int64),
                ("d_mean", C.c_void_p), ("d_rms", C.c_void_p), ("k_sigma", C.c_float),
                ("reserved", C.c_int32), ("d_cand", C.c_void_p), ("cand_cap", C.c_int64),
                ("d_ncand", C.c_void_p), ("d_plan_workspace", C.c_void_p),
                ("stream_item", C.c_void_p)]


_P = C.c_void_p
_I32, _I64, _F32, _F64 = C.c_int32, C.c_int64, C.c_float, C.c_double

# name -> (restype, argtypes); every symbol of include/dedisp.h
SIGNATURES = {
    "dd_plan_create": (C.c_int, [C.POINTER(_P), C.POINTER(_F64), _I32, _F64, C.POINTER(_F64), _I32, _I32,
                                 C.POINTER(Tuning)]),
    "dd_plan_destroy": (None, [_P]),
    "dd_plan_query": (C.c_int, [_P, _I64, C.POINTER(PlanInfo)]),
    "dd_plan_delays": (C.c_int, [_P, C.POINTER(_I32)]),
    "dd_plan_upload": (C.c_int, [_P, _P, _I64, _P]),
    "dd_dedisperse": (C.c_int, [_P, _P, _I64, _I64, _P, _I64, _P, _P, _F32, _P, _I64, _P, _P, _I64, _P]),
    "dd_dedisperse_noalloc": (C.c_int, [_P, _P, _I64, _I64, _P, _I64, _P, _P, _F32, _P, _I64, _P, _P, _P]),
    "dd_stream_create": (C.c_int, [_P, _I64, _P, _I64, _P, C.POINTER(_P)]),
    "dd_stream_push": (C.c_int, [_P, _P, _I64, _I64, _I64, _P, _I64, _P, _P, _F32, _P, _I64, _P, _P, _I64,
                                 _P, C.POINTER(_I64), C.POINTER(_I64)]),
    "dd_stream_append": (C.c_int, [_P, _P, _I64, _I64, _I64, _P, C.POINTER(_I64), C.POINTER(_I64)]),
    "dd_stream_destroy": (None, [_P]),
    "dd_batch_query": (C.c_int, [C.POINTER(BatchItem), _I32, C.POINTER(_I64)]),
    "dd_batch_dedisperse": (C.c_int, [C.POINTER(BatchItem), _I32, _P, _I64, _P]),
    "dd_detrend": (C.c_int, [_P, _I64, _I64, _I64, _I32, _P, _P]),
    "dd_boxcar": (C.c_int, [_P, _I64, _I64, _I64, _I32, _P, _I64, _P]),
    "dd_boxcar_search_workspace": (C.c_int, [_I64, _I64, C.POINTER(_I64)]),
    "dd_binned_create": (C.c_int, [C.POINTER(_P), C.POINTER(_F64), _I32, _F64, C.POINTER(_F64), _I32, _I32, _I32,
                                   C.POINTER(Tuning)]),
    "dd_binned_query": (C.c_int, [_P, _I64, C.POINTER(_I32), C.POINTER(BinnedRun), _I32, C.POINTER(_I64),
                                  C.POINTER(_F64)]),
    "dd_binned_upload": (C.c_int, [_P, _I64, _P, _I64, _P]),
    "dd_binned_dedisperse": (C.c_int, [_P, _P, _I64, _I64, _P, _I64, _P, _P, C.c_float, _P, _I64, _P, _I32, _P, _I64,
                                       _P]),
    "dd_binned_destroy": (None, [_P]),
    "dd_binned_stream_query": (C.c_int, [_P, _I64, C.POINTER(_I64), C.POINTER(_I64)]),
    "dd_binned_stream_create": (C.c_int, [_P, _I64, _P, _I64, _P, C.POINTER(_P)]),
    "dd_binned_stream_push": (C.c_int, [_P, _P, _I64, _I64, _I64, _P, _I64, _P, _P, C.c_float, _P, _I64, _P, _I32,
                                        _P, _I64, _P, C.POINTER(_I64), C.POINTER(_I64)]),
    "dd_binned_stream_set_gap_fill": (C.c_int, [_P, _I32]),
    "dd_binned_stream_destroy": (None, [_P]),
    "dd_subband_create": (C.c_int, [C.POINTER(_P), C.POINTER(_F64), _I32, _F64, C.POINTER(_F64), _I32, _I32, _I32]),
    "dd_subband_query": (C.c_int, [_P, _I64, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I32),
                                   C.POINTER(_I32)]),
    "dd_subband_upload": (C.c_int, [_P, _I64, _P, _I64, _P]),
    "dd_subband_dedisperse": (C.c_int, [_P, _P, _I64, _I64, _P, _I64, _P, _P, C.c_float, _P, _I64, _P, _I32, _P,
                                        _I64, _P]),
    "dd_subband_destroy": (None, [_P]),
    "dd_boxcar_search": (C.c_int, [_P, _I64, _I64, _I64, _P, _P, _I32, C.c_float, _P, _I64, _P, _P, _I64, _P]),
    "dd_downfactor": (C.c_int, [_P, _I32, _I64, _I64, _I64, _P, _I64, _P]),
    "dd_time_binning": (C.c_int, [_P, _I32, C.c_double, _P, _I32, _I32, _P, _P]),
    "dd_bandpass": (C.c_int, [_P, _I64, _I64, _I64, _I64, _P, _P, _P]),
    "dd_bandpass_fit": (C.c_int, [_P, _I32, _I32, _P, _P, _P]),
    "dd_rfi_clip": (C.c_int, [_P, _I64, _I64, _I64, _P, C.c_double, _I64, _P, _P, C.c_double, C.c_double, _I32,
                              _P]),
    "dd_bandpass_u8": (C.c_int, [_P, _I64, _I64, _I64, _I64, _P, _P, _P]),
    "dd_rfi_clip_u8": (C.c_int, [_P, _I64, _I64, _I64, _P, C.c_double, _I64, _P, _P, C.c_double, C.c_double, _P]),
    "dd_stream_set_gap_fill": (C.c_int, [_P, _I32]),
    "dd_candidates_check": (C.c_int, [_P, _I64, _P, C.POINTER(_I64)]),
    "dd_last_error": (C.c_char_p, []),
    "dd_version": (C.c_char_p, []),
}

_lib = None


class LibraryMissing(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Load the in-tree library; raises LibraryMissing if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise LibraryMissing(f"{path} not built: run paper_1401_8258_amd/build.py (or __graft_entry__.build())")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class DedispError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def check(code: int, allow=(DD_OK,)) -> int:
    if code in allow:
        return code
    msg = load().dd_last_error().decode(errors="replace")
    raise DedispError(code, msg or "error")
