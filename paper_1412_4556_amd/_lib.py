"""ctypes binding of libara.so (declarations mirror include/ara.h).

Argument marshalling only: every step of the trial pass runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libara.so")

ARA_OK = 0
ERRORS = {
    -1: "ARA_ERR_INVALID_ARG",
    -2: "ARA_ERR_EVENT_RANGE",
    -3: "ARA_ERR_DUP_EVENT",
    -4: "ARA_ERR_VALUE",
    -5: "ARA_ERR_OOM",
    -6: "ARA_ERR_DEVICE",
    -7: "ARA_ERR_RP",
    -8: "ARA_ERR_UNSUPPORTED",
}
ARA_FP64, ARA_FP32C = 0, 1
ARA_LAYOUT_AUTO, ARA_LAYOUT_DIRECT, ARA_LAYOUT_SPARSE, ARA_LAYOUT_COMPACT, ARA_LAYOUT_FUSED = 0, 1, 2, 3, 4
ARA_MAX_ELTS = 32
ARA_MAX_BATCH = 64
ARA_NOALLOC_MAX_SEL = 128

_P = ctypes.c_void_p
_I32, _I64, _D, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t

# name -> (restype, argtypes); the exported C-ABI of include/ara.h
SIGNATURES = {
    "ara_create_yet": (_I32, [_P, _P, _I64, _I64, _I32, _P, _P]),
    "ara_create_layer": (_I32, [_P, _I32, _P, _P, _P, _P, _P, _D, _D, _D, _D, _I32, _I32, _P]),
    "ara_run_layer": (_I32, [_P, _P, _P, _P]),
    "ara_run_layer_events": (_I32, [_P, _P, _P, _P, _P, _P]),
    "ara_run_layer_max_occurrence": (_I32, [_P, _P, _P, _P, _P]),
    "ara_run_layers": (_I32, [_P, _P, _P, _I32, _P]),
    "ara_create_batch": (_I32, [_P, _P, _I32, _P]),
    "ara_run_batch": (_I32, [_P, _P, _P]),
    "ara_batch_device_bytes": (_SZ, [_P]),
    "ara_batch_launch_config": (_I32, [_P, _P, _P]),
    "ara_batch_launch_group": (_I32, [_P, _P]),
    "ara_destroy_batch": (None, [_P]),
    "ara_batch_rebuild": (_I32, [_P, _P, _I32]),
    "ara_create_pool": (_I32, [_P, _I32, _P, _P, _P, _I32, _I32, _P]),
    "ara_destroy_pool": (None, [_P]),
    "ara_pool_device_bytes": (_SZ, [_P]),
    "ara_pool_free_slots": (_I32, [_P]),
    "ara_create_layer_from_pool": (_I32, [_P, _I32, _P, _P, _P, _D, _D, _D, _D, _P, _P]),
    "ara_pml_tvar_many": (_I32, [_P, _I32, _I64, _P, _I32, _P, _P, _P]),
    "ara_pml_tvar_many_noalloc": (_I32, [_P, _I32, _I64, _P, _I32, _P, _P, _P]),
    "ara_rollup": (_I32, [_P, _I32, _P, _I32, _I64, _P, _P]),
    "ara_pml_tvar": (_I32, [_P, _I64, _P, _I32, _P, _P, _P]),
    "ara_layer_device_bytes": (_SZ, [_P]),
    "ara_layer_layout": (_I32, [_P]),
    "ara_layer_precision": (_I32, [_P]),
    "ara_layer_n_elts": (_I32, [_P]),
    "ara_destroy_layer": (None, [_P]),
    "ara_destroy_yet": (None, [_P]),
    "ara_last_error": (ctypes.c_char_p, []),
    "ara_abi_version": (_I32, []),
}


class AraError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


_lib = None


def lib():
    """The loaded libara.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libara.so is not built ({LIB_PATH}); run paper_1412_4556_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int):
    if code != ARA_OK:
        raise AraError(code, lib().ara_last_error().decode(errors="replace"))
