"""ctypes loader of libnellox.so (the HIP library built in-tree for gfx950).

There is no fallback: if the library is missing, importing the binding's
compute entry points raises, naming the build step.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnellox.so")


class NelloxOpts(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("patch_h", ctypes.c_int32), ("patch_w", ctypes.c_int32),
                ("interleave", ctypes.c_int32)]


class NelloxImage(ctypes.Structure):
    _fields_ = [("px", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32)]


class NelloxDecodePlan(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("order", ctypes.c_int32), ("interleave", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("waves", ctypes.c_int32), ("n_lanes", ctypes.c_int64),
                ("model_hash", ctypes.c_uint64), ("ws_bytes", ctypes.c_int64), ("desc_offset", ctypes.c_int64),
                ("counter_offset", ctypes.c_int64), ("ring_offset", ctypes.c_int64), ("ring_rows", ctypes.c_int64),
                ("n_bands", ctypes.c_int64), ("progress_offset", ctypes.c_int64),
                ("band_order_offset", ctypes.c_int64)]


# exported symbol -> (restype, argtypes)
_P, _I32, _SZ, _U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_uint64
_ST = ctypes.c_int
SIGNATURES = {
    "nellox_model_create": (_ST, [_P, _SZ, ctypes.POINTER(_P)]),
    "nellox_model_destroy": (None, [_P]),
    "nellox_model_info": (_ST, [_P, _P, _P]),
    "nellox_encode_bound": (_SZ, [_I32, _I32, _P]),
    "nellox_workspace_bytes": (_SZ, [_P, _I32, _P, _P]),
    "nellox_decode_workspace_bytes": (_SZ, [_P, _I32, _P, _P]),
    "nellox_encode": (_ST, [_P, _I32, _P, _P, _P, _SZ, _P, _P, _SZ, _P]),
    "nellox_peek": (_ST, [_P, _SZ, _P, _P, _P]),
    "nellox_decode": (_ST, [_P, _I32, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "nellox_decode_trace": (_ST, [_P, _I32, _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "nellox_decode_static": (_ST, [_P, _I32, _P, _P, _P, _P, _P, _P]),
    "nellox_decode_prepare": (_ST, [_P, _I32, _P, _P, _P, _SZ, _P, _P]),
    "nellox_decode_run": (_ST, [_P, _P, _P, _P, _P, _P, _P]),
    "nellox_sample": (_ST, [_P, _I32, _P, _P, _P, _P, _SZ, _P]),
    "nellox_nll": (_ST, [_P, _I32, _P, _P, _P, _P, _P, _SZ, _P]),
    "nellox_debug_symbols": (_ST, [_P, _I32, _P, _P, _P, _P, _P, _SZ, _P]),
    "nellox_debug_cdf": (_ST, [_P, _P, _P, _P, _P, _SZ, _P]),
    "nellox_debug_check_monotone": (_ST, [_P, _P]),
    "nellox_debug_band_wait": (ctypes.c_uint64, [ctypes.c_uint64]),
    "nellox_param_count": (ctypes.c_int64, [_P]),
    "nellox_train_workspace_bytes": (_SZ, [_P, _I32, _I32, _I32]),
    "nellox_nll_fwd_train": (_ST, [_P, _P, _P, _I32, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "nellox_nll_bwd": (_ST, [_P, _P, _P, _I32, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "nellox_last_error": (ctypes.c_char_p, []),
}

STATUS_NAMES = {0: "OK", 1: "E_ARG", 2: "E_BLOB", 3: "E_CAPACITY", 4: "E_CORRUPT", 5: "E_MODEL_MISMATCH",
                6: "E_HIP", 7: "E_UNSUPPORTED"}

_lib = None


def load():
    """Load libnellox.so and declare its C signatures."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
                              "or `python paper_2201_05213_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class NelloxError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = load().nellox_last_error()
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg.decode() if msg else ''}")
        self.code = code


def check(code: int, where: str):
    if code != 0:
        raise NelloxError(code, where)
