"""ctypes loader and signatures of libfloquet.so (the C ABI in include/floquet.h).

The shared library is built in-tree by paper_2111_08044_amd.build; there is
no fallback: if it is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfloquet.so")

FL_OK, FL_EINVAL, FL_ENOMEM, FL_EHIP, FL_ESTATE, FL_ENODEV = 0, -1, -2, -3, -4, -5
FL_C64, FL_C128 = 0, 1
FL_PLAIN, FL_DENSE6_FP32, FL_DENSE6_BF16X3, FL_DENSE4_FP32 = 0, 1, 2, 3

_ERRNAMES = {FL_EINVAL: "FL_EINVAL", FL_ENOMEM: "FL_ENOMEM", FL_EHIP: "FL_EHIP",
             FL_ESTATE: "FL_ESTATE", FL_ENODEV: "FL_ENODEV"}

_lib = None

vp = C.c_void_p
dp = C.POINTER(C.c_double)
i64 = C.c_int64

SIGNATURES = {
    "fl_create": (C.c_int, [C.POINTER(vp), C.c_int, C.c_int, C.c_int, vp]),
    "fl_destroy": (C.c_int, [vp]),
    "fl_set_stream": (C.c_int, [vp, vp]),
    "fl_set_bonds": (C.c_int, [vp, dp, C.c_double]),
    "fl_set_gates": (C.c_int, [vp, dp, dp, C.c_double]),
    "fl_init_state": (C.c_int, [vp, vp, dp]),
    "fl_init_pairs": (C.c_int, [vp, vp, dp, dp]),
    "fl_apply_period": (C.c_int, [vp, vp, i64, C.c_int]),
    "fl_expect_energy": (C.c_int, [vp, vp, dp, dp]),
    "fl_expect_energy_noalloc": (C.c_int, [vp, vp, vp, vp]),
    "fl_energy_spread": (C.c_int, [vp, vp, vp, dp]),
    "fl_overlap": (C.c_int, [vp, vp, C.c_int, vp, C.c_int, dp]),
    "fl_grad_workspace_bytes": (i64, [vp]),
    "fl_grad": (C.c_int, [vp, vp, C.POINTER(vp), i64, i64, dp, C.c_int, vp, dp]),
    "fl_last_error": (C.c_char_p, []),
    "fl_xyz_bonds": (C.c_int, [C.c_int, dp, dp, dp]),
    "fl_host_gates": (C.c_int, [C.c_int, dp, C.c_double, dp]),
    "fl_host_gate_derivative": (C.c_int, [dp, dp, C.c_double, dp]),
    "fl_host_ground_states": (C.c_int, [C.c_int, dp, dp, dp]),
    "fl_xyz_generators": (C.c_int, [C.c_int, dp]),
    "fl_tile_map": (C.c_int, [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_uint64)]),
    "fl_host_window_matrix": (C.c_int, [dp, C.POINTER(C.c_int), C.c_int, C.c_int, dp, vp]),
    "fl_host_window_overlaps": (C.c_int, [dp, dp, C.POINTER(C.c_int), C.c_int, dp]),
    "fl_plan_query": (C.c_int, [C.c_int, C.c_int, C.c_int, i64, C.c_int, C.POINTER(C.c_int32), i64,
                                C.POINTER(i64)]),
}


class FloquetError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2111_08044_amd.build` "
                               "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != FL_OK:
        raise FloquetError(rc, lib().fl_last_error().decode(errors="replace"))
    return rc
