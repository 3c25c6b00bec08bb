"""ctypes view of libfft3d.so (the C ABI declared in include/fft3d.h).

Argument marshalling only.  There is no fallback: if the library is missing
the import of any entry point raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfft3d.so")

_lib = None

I64, I32, P, SZ = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t

_SIGS = {
    "fft3d_plan": (I32, [ctypes.POINTER(P), I64, I64, I64, I32, I32, I32, I32]),
    "fft3d_plan_ppb": (I32, [ctypes.POINTER(P), I64, I64, I64, I32, I32, I32, I32]),
    "fft3d_destroy": (I32, [P]),
    "fft3d_forward": (I32, [P, P, P, P]),
    "fft3d_inverse": (I32, [P, P, P, P]),
    "fft3d_backward": (I32, [P, P, P, P]),
    "fft3d_forward_noalloc": (I32, [P, P, P, P]),
    "fft3d_poisson": (I32, [P, P, P, P]),
    "fft3d_poisson_backward": (I32, [P, P, P, P]),
    "fft3d_workspace_bytes": (SZ, [P]),
    "fft3d_set_workspace": (I32, [P, P, SZ]),
    "fft3d_set_streams": (I32, [P, I32]),
    "fft3d_set_issue": (I32, [P, I32]),
    "fft3d_get_issue": (I32, [P]),
    "fft3d_set_staging": (I32, [P, I32]),
    "fft3d_get_staging": (I32, [P]),
    "fft3d_set_stage_config": (I32, [P, I32, I32, I32, I32, I32]),
    "fft3d_set_timing": (I32, [P, I32]),
    "fft3d_stage_times": (I32, [P, ctypes.POINTER(ctypes.c_float), I32]),
    "fft3d_plan_batch": (I32, [ctypes.POINTER(P), I32, ctypes.POINTER(I64), I32]),
    "fft3d_forward_batch": (I32, [P, ctypes.POINTER(P), ctypes.POINTER(P), P]),
    "fft3d_inverse_batch": (I32, [P, ctypes.POINTER(P), ctypes.POINTER(P), P]),
    "fft3d_batch_set_stage_config": (I32, [P, I64, I64, I64, I32, I32, I32, I32, I32]),
    "fft3d_batch_set_staging": (I32, [P, I64, I64, I64, I32]),
    "fft3d_batch_get_staging": (I32, [P, I64, I64, I64]),
    "fft3d_batch_set_radix_order": (I32, [P, I64, I64, I64, I32, I32]),
    "fft3d_set_radix_order": (I32, [P, I32, I32]),
    "fft3d_get_radix_order": (I32, [P, I32]),
    "fft3d_batch_set_streams": (I32, [P, I32]),
    "fft3d_batch_destroy": (I32, [P]),
    "fft3d_query_batch_placement": (I64, [I32, ctypes.POINTER(I64), I32, ctypes.POINTER(I64), I64]),
    "fft3d_status_string": (ctypes.c_char_p, [I32]),
    "fft3d_last_error": (ctypes.c_char_p, []),
    "fft3d_length_supported": (I32, [I64]),
    "fft3d_query_radix_plan": (I32, [I64, ctypes.POINTER(I32), I32]),
    "fft3d_query_twiddles": (I32, [I64, I32, P]),
    "fft3d_query_pipeline": (I64, [I64, I64, I64, I32, I32, I32, I32, I32, I32, ctypes.POINTER(I64), I64]),
    "fft3d_query_launches": (I64, [I64, I64, I64, I32, I32, I32, I32, I32, I32, ctypes.POINTER(I64), I64]),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2601_12209_amd.build` "
                "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class Fft3dError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.fft3d_status_string(status).decode()
        detail = L.fft3d_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}){': ' + detail if detail else ''}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != 0:
        raise Fft3dError(status, where)
