"""ctypes declarations of the C ABI in include/sbfwi.h (libsbfwi.so, built in-tree).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbfwi.so")

OK, EINVAL, ENOMEM, ESINGULAR, ENONFINITE, EUNSTABLE, ENOCONV, EHIP = 0, -1, -2, -3, -4, -5, -6, -7
ERROR_NAMES = {EINVAL: "SBFWI_EINVAL", ENOMEM: "SBFWI_ENOMEM", ESINGULAR: "SBFWI_ESINGULAR",
               ENONFINITE: "SBFWI_ENONFINITE", EUNSTABLE: "SBFWI_EUNSTABLE", ENOCONV: "SBFWI_ENOCONV",
               EHIP: "SBFWI_EHIP"}

vp = C.c_void_p
i64 = C.c_int64
i32 = C.c_int
dbl = C.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "sbfwi_last_error": (C.c_char_p, []),
    "sbfwi_set_allocator": (i32, [vp, vp, vp]),
    "sbfwi_build_mesh": (i32, [vp, i64, vp, vp, i64, vp, vp, dbl, C.POINTER(vp)]),
    "sbfwi_mesh_info": (i32, [vp, vp]),
    "sbfwi_factor_elements": (i32, [vp, vp, dbl, dbl, dbl, dbl, i32, i32, vp, C.POINTER(vp)]),
    "sbfwi_set_solver": (i32, [vp, dbl, i32]),
    "sbfwi_set_launch": (i32, [vp, i32, i32]),
    "sbfwi_autotune": (i32, [vp, i32, vp, vp]),
    "sbfwi_plan_bytes": (i32, [vp, i32, i64, i32, vp]),
    "sbfwi_direct_info": (i32, [vp, vp]),
    "sbfwi_direct_launches": (i32, [vp, i32, vp, i32, vp]),
    "sbfwi_copy_factor_data": (i32, [vp, i32, vp]),
    "sbfwi_coarse_pattern": (i32, [vp, vp, vp]),
    "sbfwi_forward": (i32, [vp, i32, i64, vp, vp, i32, vp, vp, i32, C.POINTER(vp), vp]),
    "sbfwi_adjoint": (i32, [vp, vp, vp, i32, vp, vp]),
    "sbfwi_gradient": (i32, [vp, vp, vp, vp, i32, vp, vp, vp]),
    "sbfwi_ckpt_info": (i32, [vp, vp]),
    "sbfwi_misfit": (i32, [vp, vp, i64, dbl, vp, vp, vp]),
    "sbfwi_factors_info": (i32, [vp, vp]),
    "sbfwi_solver_stats": (i32, [vp, vp, i32]),
    "sbfwi_fem_forward": (i32, [i32, i32, dbl, dbl, vp, dbl, dbl, i32, i64, vp, vp, i32, vp, vp, vp]),
    "sbfwi_fem_forward_noalloc": (i32, [i32, i32, dbl, dbl, vp, dbl, dbl, i32, i64, vp, vp, i32, vp, vp, vp]),
    "sbfwi_profile": (i32, [C.c_uint32]),
    "sbfwi_profile_read": (i32, [vp, i32]),
    "sbfwi_finalize": (i32, []),
    "sbfwi_destroy_mesh": (None, [vp]),
    "sbfwi_destroy_factors": (None, [vp]),
    "sbfwi_destroy_ckpt": (None, [vp]),
}

_lib = None


class SbfwiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2501_06748_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code: int):
    if code != OK:
        raise SbfwiError(code, lib().sbfwi_last_error().decode())
