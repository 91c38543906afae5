"""Host timing baseline: the paper's Gray-code brute force (Algorithm 1 with
the Sec. 3.1 prefix split, float64, OpenMP) -- test infrastructure only.

Used by the benchmark to time the paper's own method on the host cores beside
the oracle, and by the CPU tests, which check it against the oracle.  The C
source is ``gray_cpu.c`` next to this file, built by ``build.py``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# QUBO_GRAY_LIB: another build of the same library (the sanitizer run of the CPU tests)
LIB_PATH = os.environ.get("QUBO_GRAY_LIB") or os.path.join(_HERE, "libqubo_gray_cpu.so")

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _build

        _build.build_gray()
    lib = ctypes.CDLL(LIB_PATH)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.qg_min_f32.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                               u64p, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_double), u64p]
    lib.qg_min_f32.restype = ctypes.c_int
    lib.qg_max_threads.argtypes = []
    lib.qg_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def max_threads() -> int:
    return _load().qg_max_threads()


def minimum(Q, m: int, prefixes=None, threads: int = 0):
    """(energy float64, mask int) of the lowest state whose top m bits are one
    of `prefixes` (every prefix when None); ties go to the lower mask."""
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    if Q.ndim != 2 or Q.shape[0] != Q.shape[1]:
        raise ValueError("Q must be square")
    n = Q.shape[0]
    lib = _load()
    e = ctypes.c_double()
    mk = ctypes.c_uint64()
    if prefixes is None:
        pp, cnt = None, 0
    else:
        arr = np.ascontiguousarray(np.asarray(prefixes, dtype=np.uint64))
        pp, cnt = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), arr.size
    rc = lib.qg_min_f32(Q.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, n, m, pp, cnt, threads,
                        ctypes.byref(e), ctypes.byref(mk))
    if rc != 0:
        raise ValueError(f"qg_min_f32: invalid arguments (n={n}, m={m})")
    return e.value, int(mk.value)
