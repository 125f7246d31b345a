"""ctypes loader for libndft.so (the C ABI declared in include/ndft.h).

Loading fails loudly when the library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libndft.so")

# Every symbol include/ndft.h declares, with its ctypes signature.
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_SZ = ctypes.c_size_t
_ST = ctypes.c_int

SIGNATURES = {
    "ndft_forward_workspace": (_SZ, [_I64, _I64, _I64, _I64, _I32]),
    "ndft_forward": (_ST, [_P, _P, _I64, _I64, _I64, _I64, _I32, _P, _SZ, _P]),
    "ndft_caf_workspace": (_SZ, [_I64, _I64, _I64, _I64, _I64, _I32]),
    "ndft_caf": (_ST, [_P, _P, _I64, _I64, _I64, _I64, _I64, _P, _I32, _P, _SZ, _P]),
    "ndft_caf_noalloc": (_ST, [_P, _P, _I64, _I64, _I64, _I64, _I64, _P, _I32, _P]),
    "ndft_nfft_workspace": (_SZ, [_I64, _I64]),
    "ndft_nfft": (_ST, [_P, _P, _I64, _I64, _I32, _P, _SZ, _P]),
    "ndft_caf12b_workspace": (_SZ, [_I64, _I64, _I64, _I64, _I64, _I32]),
    "ndft_caf12b": (_ST, [_P, _P, _I64, _I64, _I64, _I64, _I64, _P, _I32, _P, _SZ, _P]),
    "ndft_caf12c_workspace": (_SZ, [_I64, _I64, _I64, _I64, _I64, _I32]),
    "ndft_caf12c": (_ST, [_P, _P, _I64, _I64, _I64, _I64, _I64, _P, _I32, _P, _SZ, _P]),
    "ndft_caf_batched_workspace": (_SZ, [_P, _I32, _I32, _I32]),
    "ndft_caf_batched_prepare": (_ST, [_P, _I32, _I32, _I32, _P, _SZ, _P]),
    "ndft_caf_batched": (_ST, [_P, _P, _P, _P, _P, _SZ, _P]),
    "ndft_caf_batched_dev_workspace": (_SZ, [_I32, _I64, _I64, _I64, _I32]),
    "ndft_caf_batched_dev": (_ST, [_P, _P, _P, _P, _I32, _I32, _P, _SZ, _P]),
    "ndft_caf_batched_dev_status": (_ST, [_P, _P, _P]),
    "ndft_caf_backward_workspace": (_SZ, [_I64, _I64, _I64, _I64, _I64, _I32]),
    "ndft_caf_backward": (_ST, [_P, _P, _I64, _I64, _I64, _I64, _I64, _P, _P, _P, _I32, _P, _SZ, _P]),
    "ndft_dbg_signs": (_ST, [_P, _P, _I64, _I64, _I64, _I64, _I64, _P, _P, _P]),
    "ndft_dbg_split": (_ST, [_P, _P, _I64, _I64, _I64, _I64, _I64, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "ndft_dbg_fast_tables": (_I32, [_I32]),
    "ndft_plan_count": (_I32, [_I32]),
    "ndft_plan_name": (ctypes.c_char_p, [_I32, _I32]),
    "ndft_set_plan": (_ST, [_I32, _I32, _I32]),
    "ndft_get_plan": (_ST, [_I32, _I64, _I64, _I64, _I64, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "ndft_prof_enable": (_ST, [_I32]),
    "ndft_prof_read": (_ST, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)]),
    "ndft_prof_read_slot": (_ST, [_I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)]),
    "ndft_status_string": (ctypes.c_char_p, [_ST]),
    "ndft_version": (ctypes.c_char_p, []),
}


class NdftCpi(ctypes.Structure):
    """Mirror of ndft_cpi."""

    _fields_ = [(name, ctypes.c_int64) for name in
                ("n", "surv_off", "ref_off", "out_off", "tau0", "n_tau", "p0", "n_dop")]


class NdftBatch(ctypes.Structure):
    """Mirror of ndft_batch (host description of a prepared batch)."""

    _fields_ = [(name, ctypes.c_int32) for name in
                ("prec", "plan", "n_cpi", "n_items", "grid", "table_bytes", "max_red_blocks",
                 "max_prep_blocks")] + [("tag", ctypes.c_uint64), ("ws_bytes", ctypes.c_uint64)]


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libndft.so is not built (expected at %s); run "
                "`python -m paper_1402_0532_amd.build` or __graft_entry__.build()" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def status_string(st: int) -> str:
    return load().ndft_status_string(st).decode()


def check(st: int, what: str = "ndft") -> None:
    if st != 0:
        raise RuntimeError("%s: %s" % (what, status_string(st)))
