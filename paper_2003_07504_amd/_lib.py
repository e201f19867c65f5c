"""ctypes loader for libils.so (the HIP library built from csrc/).

Loading fails loudly when the library has not been built: there is no
fallback implementation."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libils.so")

c_float_p = ctypes.POINTER(ctypes.c_float)


class IlsFrame(ctypes.Structure):
    """Mirror of struct ils_frame (include/ils.h)."""
    _fields_ = [
        ("f", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("H", ctypes.c_int),
        ("W", ctypes.c_int),
        ("C", ctypes.c_int),
        ("lam", ctypes.c_float),
        ("p", ctypes.c_float),
        ("eps", ctypes.c_float),
        ("N", ctypes.c_int),
        ("u0", ctypes.c_void_p),
        ("penalty", ctypes.c_int),
        ("gamma", ctypes.c_float),
    ]


PENALTY_CHARBONNIER = 0
PENALTY_WELSCH = 1


# name -> (restype, argtypes); exactly the functions include/ils.h declares.
SIGNATURES = {
    "ils_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ils_length_supported": (ctypes.c_int, [ctypes.c_int]),
    "ils_size_supported": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
    "ils_check_args": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_int]),
    "ils_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int] * 4),
    "ils_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(IlsFrame), ctypes.c_int]),
    "ils_plan_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p, ctypes.c_uint]),
    "ils_plan_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "ils_plan_set_persistent": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "ils_plan_set_wait_limit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_longlong]),
    "ils_smooth": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_int, ctypes.c_void_p]),
    "ils_smooth_welsch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_int,
                                         ctypes.c_void_p]),
    "ils_detail_enhance": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                          ctypes.c_int, ctypes.c_float, ctypes.c_void_p]),
    "ils_luminance_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int]),
    "ils_smooth_luminance": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int,
                                            ctypes.c_float, ctypes.c_void_p]),
    "ils_tone_map": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_void_p]),
    "ils_tone_map_multiscale_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "ils_tone_map_multiscale": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                               c_float_p, c_float_p, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                               ctypes.c_int, ctypes.c_float, ctypes.c_void_p]),
    "ils_energy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_void_p]),
    "ils_energy_welsch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_void_p]),
    "ils_iterate_from_c": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                          ctypes.c_float, ctypes.c_float, ctypes.c_int, ctypes.c_void_p]),
    "ils_iterate_from": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float, ctypes.c_int, ctypes.c_void_p]),
    "ils_smooth_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(IlsFrame), ctypes.c_int]),
    "ils_rms_diff": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                    ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_longlong),
                                    ctypes.c_int, ctypes.c_void_p]),
    "ils_profile_begin": (ctypes.c_int, [ctypes.c_void_p]),
    "ils_profile_end": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int)]),
    "ils_enqueue_pass": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float]),
    "ils_noalloc_max_bytes": (ctypes.c_size_t, []),
    "ils_smooth_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                                          ctypes.c_float, ctypes.c_float, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "ils_last_error": (ctypes.c_int, [ctypes.c_void_p]),
    "ils_shape_variants": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int)]),
    "ils_plan_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "ils_plan_set_shapes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int]),
    "ils_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ils_debug_rhs_spectrum": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                              ctypes.c_float, ctypes.c_void_p]),
    "ils_debug_column_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                              ctypes.c_void_p]),
    "ils_debug_row_inverse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_void_p]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libils.so once and attach the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_2003_07504_amd.build, or __graft_entry__.build()).")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class IlsError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = load().ils_status_string(status).decode()
        super().__init__(f"{what}: {msg} (status {status})" if what else f"{msg} (status {status})")


def check(status: int, what: str = "") -> None:
    if status != 0:
        raise IlsError(status, what)
