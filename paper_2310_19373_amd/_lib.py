"""ctypes binding of ``libqubo_bf.so`` (the C ABI declared in include/qubo_bf.h).

Argument marshalling only: every step of the enumeration runs in the HIP
library.  Loading fails loudly when the library has not been built; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# QUBO_BF_LIB: another build of the same library (the sanitizer run of the CPU tests)
LIB_PATH = os.environ.get("QUBO_BF_LIB") or os.path.join(_HERE, "libqubo_bf.so")

QUBO_F32 = 0
QUBO_I32 = 1
QUBO_F64 = 2
QUBO_I64 = 3

QUBO_OK = 0
QUBO_ERR_INVALID_ARG = -1
QUBO_ERR_NONFINITE = -2
QUBO_ERR_WORKSPACE = -3
QUBO_ERR_HIP = -4
QUBO_ERR_UNCERTAIN = -5
QUBO_ERR_RANGE = -6
QUBO_ERR_OVERFLOW = -7

TUNE_SINGLE_OUTER_BITS = 1
TUNE_SINGLE_UNIT_BITS = 2
TUNE_BATCHED_OUTER_BITS = 3
TUNE_WAVES_PER_CU = 4
TUNE_KPRIME = 5
TUNE_CHUNK_SINGLE = 6
TUNE_CHUNK_BATCHED = 7
TUNE_DYNAMIC_QUEUE = 8
TUNE_LOGZ_FACTORED = 9
TUNE_SEED_SWEEPS = 10
TUNE_HALF_SCREEN = 11

# size of the static workspace array of qubo_bf_solve_noalloc (QUBO_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 16 << 20

# Every symbol include/qubo_bf.h declares: name -> (restype, argtypes)
_vp, _sz, _i, _i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int64
SIGNATURES = {
    "qubo_bf_workspace_size": (_sz, [_i, _i, _i]),
    "qubo_bf_solve": (_i, [_vp, _i, _i64, _i, _i, _vp, _vp, _vp, _vp, _sz, _vp]),
    "qubo_bf_workspace_size_kp": (_sz, [_i, _i, _i, _i]),
    "qubo_bf_solve_kp": (_i, [_vp, _i, _i64, _i, _i, _i, _vp, _vp, _vp, _vp, _sz, _vp]),
    "qubo_bf_solve_noalloc": (_i, [_vp, _i, _i64, _i, _i, _vp, _vp, _vp, _vp]),
    "qubo_bf_batched_workspace_size": (_sz, [_i, _i, _i, _i]),
    "qubo_bf_range_workspace_size": (_sz, [_i, _i, _i, _i]),
    "qubo_bf_solve_range": (_i, [_vp, _i, _i64, _i, _i, _i, _i64, _i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "qubo_bf_merge_topk": (_i, [_i, _i, _vp, _vp, _i, _i, _vp, _vp, _vp]),
    "qubo_bf_solve_batched": (_i, [_i, _vp, _i, _vp, _i, _i, _vp, _vp, _vp, _vp, _sz, _vp]),
    "qubo_logz_workspace_size": (_sz, [_i, _i]),
    "qubo_logz_fwd": (_i, [_i, _vp, _i, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "qubo_logz_bwd": (_i, [_i, _vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "qubo_logz_moments": (_i, [_i, _vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "qubo_logz_sample_workspace_size": (_sz, [_i, _i]),
    "qubo_logz_sample": (_i, [_i, _vp, _i, _vp, _vp, _i, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "qubo_last_error": (ctypes.c_char_p, []),
    "qubo_version": (ctypes.c_char_p, []),
    "qubo_bf_set_tuning": (_i, [_i, _i]),
    "qubo_bf_get_tuning": (_i, [_i]),
    "qubo_prof_enable": (_i, [_i]),
    "qubo_prof_collect": (_i, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
}

_lib = None


class QuboError(RuntimeError):
    """A non-OK return or device status of the HIP library."""

    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def lib():
    """The loaded library (raises if it is missing: build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_2310_19373_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    return lib().qubo_last_error().decode()


def check(rc: int):
    if rc != QUBO_OK:
        raise QuboError(rc, last_error())


def set_tuning(knob: int, value: int):
    check(lib().qubo_bf_set_tuning(knob, value))


def get_tuning(knob: int) -> int:
    return lib().qubo_bf_get_tuning(knob)


def prof_enable(on: bool):
    check(lib().qubo_prof_enable(1 if on else 0))


def prof_collect(name: str):
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    check(lib().qubo_prof_collect(name.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value
