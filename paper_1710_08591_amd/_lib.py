"""ctypes binding of libfftbf.so (argument marshalling only).

Every function of the C ABI in include/fftbf.h is bound here under its own
name.  All compute runs in the library's HIP kernels; this module never
falls back to anything else and raises if the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfftbf.so")

BF_OK = 0
BF_ERR_INVALID_ARGUMENT = -1
BF_ERR_UNSUPPORTED = -2
BF_ERR_OUT_OF_MEMORY = -3
BF_ERR_DEVICE = -4
BF_ERR_REJECTED = -5
BF_ERR_EVICTED = -6
BF_ERR_NOT_READY = -7

BF_PREC_FP32 = 0
BF_PREC_FP16_MFMA = 1
BF_PREC_FP8_MFMA = 2

BF_OUT_INTENSITY = 0
BF_OUT_COMPLEX = 1


class bf_plan_desc(C.Structure):
    _fields_ = [
        ("n_ew", C.c_int32), ("n_ns", C.c_int32), ("m_ew", C.c_int32), ("m_ns", C.c_int32),
        ("n_pol", C.c_int32), ("n_chan", C.c_int32), ("block", C.c_int32),
        ("n_ns_keep", C.c_int32), ("pol_sum", C.c_int32), ("precision", C.c_int32),
        ("d_over_lambda", C.POINTER(C.c_double)), ("ns_select", C.POINTER(C.c_int32)),
    ]


class bf_server_stats(C.Structure):
    _fields_ = [
        ("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
        ("evicted", C.c_int64), ("in_flight", C.c_int64), ("budget_used", C.c_int64),
        ("tiles_done", C.c_int64), ("launches", C.c_int64),
    ]


_P = C.c_void_p
_SIGS = {
    "bf_version": (C.c_char_p, []),
    "bf_status_string": (C.c_char_p, [C.c_int32]),
    "bf_last_error": (C.c_char_p, []),
    "bf_plan_create": (C.c_int32, [C.POINTER(bf_plan_desc), C.POINTER(_P)]),
    "bf_plan_destroy": (C.c_int32, [_P]),
    "bf_plan_get_desc": (C.c_int32, [_P, C.POINTER(bf_plan_desc)]),
    "bf_beamform_fft": (C.c_int32, [_P, _P, C.c_int64, _P, C.c_int32, _P, _P]),
    "bf_beamform_fft_gains": (C.c_int32, [_P, _P, C.c_int64, _P, C.c_int32, _P, _P]),
    "bf_form_tied_beams": (C.c_int32, [_P, _P, C.c_int64, C.c_int32, C.c_int32, _P, C.c_int32,
                                       C.c_int32, _P, _P]),
    "bf_form_tied_beams_v": (C.c_int32, [_P, _P, C.c_int64, _P, C.c_int32, C.c_int32, _P, C.c_int32,
                                         _P, _P]),
    "bf_tied_workspace_size": (C.c_size_t, [_P, C.c_int32, C.c_int64]),
    "bf_form_tied_beams_v_ws": (C.c_int32, [_P, _P, C.c_int64, _P, C.c_int32, C.c_int32, _P, C.c_int32,
                                            _P, C.c_size_t, _P, _P]),
    "bf_form_tied_beams_v_noalloc": (C.c_int32, [_P, _P, C.c_int64, _P, C.c_int32, C.c_int32, _P, C.c_int32,
                                                 _P, _P]),
    "bf_accumulate_intensity": (C.c_int32, [_P, C.c_int64, C.c_int64, C.c_int32, C.c_int32, _P, _P]),
    "bf_regrid_create": (C.c_int32, [_P, _P, C.c_int32, _P, C.c_int32, C.POINTER(_P)]),
    "bf_regrid_create_2d": (C.c_int32, [_P, _P, C.c_int32, C.POINTER(_P)]),
    "bf_regrid_destroy": (C.c_int32, [_P]),
    "bf_localize": (C.c_int32, [_P, _P, C.c_int64, C.c_int32, C.c_int32, _P, _P, _P]),
    "bf_regrid_intensity": (C.c_int32, [_P, _P, C.c_int64, _P, _P]),
}
_SIGS.update({
    "bf_server_create": (C.c_int32, [_P, C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.POINTER(_P)]),
    "bf_server_destroy": (C.c_int32, [_P]),
    "bf_server_ring": (C.c_int32, [_P, C.POINTER(_P), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "bf_server_advance": (C.c_int32, [_P, C.c_int64, _P, C.c_int32, _P]),
    "bf_server_submit": (C.c_int32, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int64, _P, C.c_double,
                                     C.POINTER(C.c_int64)]),
    "bf_server_pump": (C.c_int32, [_P]),
    "bf_server_poll": (C.c_int32, [_P, C.c_int64, C.POINTER(C.c_double)]),
    "bf_server_result": (C.c_int32, [_P, C.c_int64, C.POINTER(_P), C.POINTER(C.c_int64)]),
    "bf_server_copy_result": (C.c_int32, [_P, C.c_int64, _P, _P]),
    "bf_server_release": (C.c_int32, [_P, C.c_int64]),
    "bf_server_cancel": (C.c_int32, [_P, C.c_int64]),
    "bf_server_stats_get": (C.c_int32, [_P, C.POINTER(bf_server_stats)]),
    "bf_server_now": (C.c_double, [_P]),
})
_OPTIONAL = {}


class LibraryMissing(RuntimeError):
    pass


_lib = None


def lib() -> C.CDLL:
    """Load libfftbf.so (built in-tree); raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is not built: run `python -m paper_1710_08591_amd.build`")
    l = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(l, name)
        f.restype = res
        f.argtypes = args
    for name, (res, args) in _OPTIONAL.items():
        f = getattr(l, name, None)
        if f is not None:
            f.restype = res
            f.argtypes = args
    _lib = l
    return l


def declared_symbols() -> list:
    """Function names declared in the public headers (include/*.h)."""
    import glob
    import re
    root = os.path.dirname(HERE)
    names = []
    for h in sorted(glob.glob(os.path.join(root, "include", "*.h"))):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"\b(bf_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


class BFError(RuntimeError):
    def __init__(self, status: int, where: str):
        l = lib()
        detail = l.bf_last_error().decode()
        super().__init__(f"{where}: {l.bf_status_string(status).decode()} ({status}): {detail}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != BF_OK:
        raise BFError(status, where)
