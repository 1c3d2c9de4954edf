"""ctypes declarations of the libozemu C-ABI (include/ozemu.h).

Loading fails loudly when the library has not been built: there is no CPU
fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libozemu.so")

OZEMU_OK = 0
OZEMU_ERR_INVALID_ARG = -1
OZEMU_ERR_K_TOO_LARGE = -2
OZEMU_ERR_UNSUPPORTED = -3
OZEMU_ERR_WORKSPACE = -4
OZEMU_ERR_HIP = -5

OZEMU_INT8 = 0
FORMATS = {"INT8": 0, "E4M3": 1, "E2M3": 2, "E2M1": 3}
SCALING = {"F53": 0, "W": 1, "G": 2}
SHIFT_NONFINITE = -(2 ** 31)

_i64 = C.c_int64
_vp = C.c_void_p
_st = C.c_int

# name -> (restype, argtypes), exactly as declared in include/ozemu.h
SIGNATURES = {
    "ozemu_plan_create": (_st, [C.POINTER(_vp), C.c_int, C.c_int, C.c_int]),
    "ozemu_plan_create_moduli": (_st, [C.POINTER(_vp), C.c_int, C.c_int,
                                       C.POINTER(C.c_int32), C.c_int]),
    "ozemu_plan_create_fp": (_st, [C.POINTER(_vp), C.c_int, C.c_int, _i64, C.c_int]),
    "ozemu_plan_channels": (_st, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_int)]),
    "ozemu_plan_destroy": (_st, [_vp]),
    "ozemu_plan_moduli": (_st, [_vp, C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_int)]),
    "ozemu_plan_kept_bits": (_st, [_vp, _i64, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "ozemu_plan_k_max": (_st, [_vp, C.POINTER(_i64)]),
    "ozemu_plane_dims": (_st, [_vp, _i64, _i64, _i64, C.POINTER(_i64), C.POINTER(_i64),
                               C.POINTER(_i64)]),
    "ozemu_workspace_size": (_st, [_vp, _i64, _i64, _i64, C.POINTER(C.c_size_t)]),
    "ozemu_dgemm": (_st, [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp,
                          C.c_size_t]),
    "ozemu_blocked_workspace_size": (_st, [_vp, _i64, _i64, _i64, _i64,
                                           C.POINTER(C.c_size_t)]),
    "ozemu_dgemm_blocked": (_st, [_vp, _vp, _i64, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp,
                                  _i64, _vp, C.c_size_t]),
    "ozemu_scale": (_st, [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _vp,
                          C.c_size_t]),
    "ozemu_reduce": (_st, [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _vp,
                           _vp]),
    "ozemu_residue_gemm": (_st, [_vp, _vp, _i64, _i64, _i64, _vp, _vp, _vp]),
    "ozemu_reconstruct": (_st, [_vp, _vp, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _i64]),
    "ozemu_dgemm_fwd_cache": (_st, [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp,
                                    _i64, _vp, _vp, _vp, _vp, _vp, C.c_size_t]),
    "ozemu_bwd_workspace_size": (_st, [_vp, _i64, _i64, _i64, C.POINTER(C.c_size_t)]),
    "ozemu_dgemm_bwd": (_st, [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp,
                              _i64, _vp, _i64, _vp, C.c_size_t]),
    "ozemu_group_create": (_st, [C.POINTER(_vp), C.c_int, C.POINTER(_vp), C.POINTER(_i64),
                                 C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_vp),
                                 C.POINTER(_i64), C.POINTER(_vp), C.POINTER(_i64),
                                 C.POINTER(_vp), C.POINTER(_i64)]),
    "ozemu_group_workspace_size": (_st, [_vp, C.POINTER(C.c_size_t)]),
    "ozemu_group_run": (_st, [_vp, _vp, _vp, C.c_size_t]),
    "ozemu_group_destroy": (_st, [_vp]),
    "ozemu_status_string": (C.c_char_p, [C.c_int]),
    "ozemu_last_error": (C.c_char_p, []),
    "ozemu_version": (C.c_char_p, []),
}

_lib = None


class OzemuError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (status_name(status), message))
        self.status = status


def load():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libozemu.so is not built; run `python -m paper_2609_37693_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def status_name(status: int) -> str:
    return load().ozemu_status_string(status).decode()


def check(status: int):
    if status != OZEMU_OK:
        raise OzemuError(status, load().ozemu_last_error().decode())
