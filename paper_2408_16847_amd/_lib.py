"""ctypes loader of libzeta3.so (the C ABI declared in include/zeta3.h)."""

from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  -- loads the HIP runtime that libzeta3 shares with torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libzeta3.so")

_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_D = ctypes.c_double

# name -> (restype, argtypes); every symbol declared in include/zeta3.h
SIGNATURES = {
    "z3_build_index": (_I, [_I64, _P, _P, _I, _P, _D, _P, ctypes.POINTER(_P)]),
    "z3_build_index_planar": (_I, [_I64, _P, _P, _I, _P, _D, _P, ctypes.POINTER(_P)]),
    "z3_index_set_values": (_I, [_P, _I, _P, _P]),
    "z3_index_info": (_I, [_P, _P, _P, _P, _P, _P]),
    "z3_index_update_values": (_I, [_P, _P, _P]),
    "z3_index_prepare_capture": (_I, [_P, ctypes.c_size_t, _P]),
    "z3_index_perm": (_I, [_P, _P, _P]),
    "z3_index_set_batch_shape": (_I, [_P, _I, _I]),
    "z3_index_batch_shape": (_I, [_P, _I, _I, _P, _P]),
    "z3_index_free": (None, [_P]),
    "z3_accumulate_multipoles": (_I, [_P, _I, _I, _I, _I, _I64, _I64, _P, _P, _P, _P, _P, _P]),
    "z3_contract": (_I, [_I64, _I, _I, _I, _P, _P, _P, _P]),
    "z3_estimate": (_I, [_P, _I, _I, _I, _I64, _I64, _P, _P, _P]),
    "z3_estimate_ex": (_I, [_P, _I, _I, _I, ctypes.c_uint, _I64, _I64, _P, _P, _P]),
    "z3_estimate_static": (_I, [_P, _I, _I, _I, ctypes.c_uint, _I64, _I64, _P, _P, _P]),
    "z3_index_set_phi_bins": (_I, [_P, _I, _P]),
    "z3_accumulate_histogram": (_I, [_P, _I, _I, _I, _I, _I64, _I64, _P, _P, _P, _P, _P, _P]),
    "z3_estimate_histogram": (_I, [_P, _I, _I, _I, _I64, _I64, _P, _P, _P]),
    "z3_estimate_cross": (_I, [_P, _I, _I, _I, _I, _I, _I, _I64, _I64, _P, _P, _P]),
    "z3_estimate_cross_catalogues": (_I, [_P, _I, _P, _I, _I64, _P, _P, _P, _I, _I, _I64, _I64, _P, _P, _P, _P,
                                          _P]),
    "z3_adjoint": (_I, [_P, _I, _I, _I64, _I64, _P, _D, _P, _P]),
    "z3_adjoint_maps": (_I, [_P, _I, _I64, _I64, _P, _D, _P, _P]),
    "z3_estimate_maps": (_I, [_P, _I, _I, _I64, _I64, _P, _P, _P]),
    "z3_estimate_pivots": (_I, [_P, _I, _I64, _P, _P, _P, _I, _I, _I64, _I64, _P, _P, _P, _P]),
    "z3_pivot_weight_sum": (_I, [_P, _I64, _I64, _P, _P]),
    "z3_finalize": (_I, [_I, _I, _I, _P, _P, _P]),
    "z3_resum": (_I, [_I, _I, _P, _I, _P, _P, _P]),
    "z3_fftlog_workspace_size": (_I, [_I, _I, _I, _I, _P]),
    "z3_fftlog_a_functions": (_I, [_I, _P, _D, _D, _P, _I, _D, _D, _I, _P, _I, _P, _P, _P, ctypes.c_size_t, _P]),
    "z3_set_device_alloc_limit": (_I, [ctypes.c_size_t]),
    "z3_sync": (_I, [_P]),
    "z3_status_string": (ctypes.c_char_p, [_I]),
    "z3_last_error": (ctypes.c_char_p, []),
    "z3_profile_enable": (_I, [_I]),
    "z3_profile_read": (_I, [_P, _P, _I]),
}

_lib = None


class Zeta3Error(RuntimeError):
    def __init__(self, status: int, fn: str, detail: str):
        super().__init__(f"{fn} failed with status {status}: {detail}")
        self.status = status


def load():
    """Load libzeta3.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libzeta3.so not found at {LIB_PATH}; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def call(name: str, *args) -> None:
    lib = load()
    st = getattr(lib, name)(*args)
    if st != 0:
        raise Zeta3Error(st, name, lib.z3_last_error().decode(errors="replace"))
