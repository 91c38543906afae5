"""CPU oracle (test infrastructure only).

Plain, slow, obviously correct evaluation of the QUBO objective of Eq. 1 in
natural binary order, in float64 (float32 / float64 Q) or int64 (int32 / int64
Q), plus the log-partition function and its gradient defined directly from
their sums.
Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package; the product path never does.  It shares no code with the HIP
library; the only common module is the seeded input generator.

The C source is ``qubo_oracle.c`` next to this file, built by ``build.py``
with gcc (OpenMP, -O2, -ffp-contract=off) into ``libqubo_oracle.so``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# QUBO_ORACLE_LIB: another build of the same library (the sanitizer run of the CPU tests)
LIB_PATH = os.environ.get("QUBO_ORACLE_LIB") or os.path.join(_HERE, "libqubo_oracle.so")

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _build

        _build.build()
    lib = ctypes.CDLL(LIB_PATH)
    c_f = ctypes.POINTER(ctypes.c_float)
    c_i = ctypes.POINTER(ctypes.c_int32)
    c_d = ctypes.POINTER(ctypes.c_double)
    c_u = ctypes.POINTER(ctypes.c_uint64)
    c_l = ctypes.POINTER(ctypes.c_int64)
    i64, u64 = ctypes.c_int64, ctypes.c_uint64
    lib.qo_energy_f32.argtypes = [c_f, ctypes.c_int, i64, u64]
    lib.qo_energy_f32.restype = ctypes.c_double
    lib.qo_energy_i32.argtypes = [c_i, ctypes.c_int, i64, u64]
    lib.qo_energy_i32.restype = ctypes.c_int64
    lib.qo_energies_f32.argtypes = [c_f, ctypes.c_int, i64, c_u, i64, c_d]
    lib.qo_energies_f32.restype = None
    lib.qo_energies_i32.argtypes = [c_i, ctypes.c_int, i64, c_u, i64, c_l]
    lib.qo_energies_i32.restype = None
    lib.qo_topk_f32.argtypes = [c_f, ctypes.c_int, i64, u64, u64, ctypes.c_int, c_d, c_u, ctypes.c_int]
    lib.qo_topk_f32.restype = ctypes.c_int
    lib.qo_topk_i32.argtypes = [c_i, ctypes.c_int, i64, u64, u64, ctypes.c_int, c_l, c_u, ctypes.c_int]
    lib.qo_topk_i32.restype = ctypes.c_int
    lib.qo_energy_f64.argtypes = [c_d, ctypes.c_int, i64, u64]
    lib.qo_energy_f64.restype = ctypes.c_double
    lib.qo_energy_i64.argtypes = [c_l, ctypes.c_int, i64, u64]
    lib.qo_energy_i64.restype = ctypes.c_int64
    lib.qo_energies_f64.argtypes = [c_d, ctypes.c_int, i64, c_u, i64, c_d]
    lib.qo_energies_f64.restype = None
    lib.qo_energies_i64.argtypes = [c_l, ctypes.c_int, i64, c_u, i64, c_l]
    lib.qo_energies_i64.restype = None
    lib.qo_topk_f64.argtypes = [c_d, ctypes.c_int, i64, u64, u64, ctypes.c_int, c_d, c_u, ctypes.c_int]
    lib.qo_topk_f64.restype = ctypes.c_int
    lib.qo_topk_i64.argtypes = [c_l, ctypes.c_int, i64, u64, u64, ctypes.c_int, c_l, c_u, ctypes.c_int]
    lib.qo_topk_i64.restype = ctypes.c_int
    lib.qo_logz_f32.argtypes = [c_f, ctypes.c_int, i64, ctypes.c_double, c_d, ctypes.c_int]
    lib.qo_logz_f32.restype = ctypes.c_double
    lib.qo_grad_f32.argtypes = [c_f, ctypes.c_int, i64, ctypes.c_double, ctypes.c_double, c_d, ctypes.c_int]
    lib.qo_grad_f32.restype = ctypes.c_int
    lib.qo_max_threads.argtypes = []
    lib.qo_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _prep(Q):
    Q = np.ascontiguousarray(Q)
    if Q.ndim != 2 or Q.shape[0] != Q.shape[1]:
        raise ValueError("Q must be square")
    if Q.dtype == np.float32:
        return Q, True
    if Q.dtype == np.int32:
        return Q, False
    raise TypeError("Q must be float32 or int32")


# element type -> (C element, C result, result dtype, name suffix, sentinel)
_KINDS = {
    np.dtype(np.float32): (ctypes.c_float, ctypes.c_double, np.float64, "f32"),
    np.dtype(np.int32): (ctypes.c_int32, ctypes.c_int64, np.int64, "i32"),
    np.dtype(np.float64): (ctypes.c_double, ctypes.c_double, np.float64, "f64"),
    np.dtype(np.int64): (ctypes.c_int64, ctypes.c_int64, np.int64, "i64"),
}


def _kind(Q):
    Q = np.ascontiguousarray(Q)
    if Q.ndim != 2 or Q.shape[0] != Q.shape[1]:
        raise ValueError("Q must be square")
    if Q.dtype not in _KINDS:
        raise TypeError("Q must be float32, int32, float64 or int64")
    return Q, _KINDS[Q.dtype]


def max_threads() -> int:
    return _load().qo_max_threads()


def energy(Q, mask: int):
    """f_Q(x) for the mask (bit i = x_i): float (f64) or int (int64)."""
    Q, (ce, _, _, sfx) = _kind(Q)
    lib = _load()
    n = Q.shape[0]
    return getattr(lib, "qo_energy_" + sfx)(_ptr(Q, ce), n, n, mask)


def energies(Q, masks):
    Q, (ce, cr, rt, sfx) = _kind(Q)
    lib = _load()
    n = Q.shape[0]
    m = np.ascontiguousarray(np.asarray(masks, dtype=np.uint64))
    out = np.empty(m.shape, dtype=rt)
    getattr(lib, "qo_energies_" + sfx)(_ptr(Q, ce), n, n, _ptr(m, ctypes.c_uint64), m.size, _ptr(out, cr))
    return out


def topk(Q, k: int, lo: int = 0, hi: int | None = None, threads: int = 0):
    """The k lowest (energy, mask) pairs over masks in [lo, hi), natural order.

    Returns (energies float64|int64 [k], masks uint64 [k]); missing slots carry
    +inf / INT64_MAX and mask 2^64-1.
    """
    Q, (ce, cr, rt, sfx) = _kind(Q)
    lib = _load()
    n = Q.shape[0]
    if hi is None:
        hi = 1 << n
    M = np.empty(k, dtype=np.uint64)
    E = np.empty(k, dtype=rt)
    rc = getattr(lib, "qo_topk_" + sfx)(_ptr(Q, ce), n, n, lo, hi, k, _ptr(E, cr), _ptr(M, ctypes.c_uint64),
                                         threads)
    if rc != 0:
        raise ValueError("oracle topk: bad arguments")
    return E, M


def logz(Q, beta: float, threads: int = 0, with_mean: bool = False):
    """log sum_x exp(-beta f(x)) in float64 (float Q only)."""
    Q, isf = _prep(Q)
    if not isf:
        Q = Q.astype(np.float32)
    lib = _load()
    mean = ctypes.c_double(0.0)
    v = lib.qo_logz_f32(_ptr(Q, ctypes.c_float), Q.shape[0], Q.shape[0], float(beta),
                        ctypes.byref(mean), threads)
    return (v, mean.value) if with_mean else v


def grad(Q, beta: float, logz_value: float | None = None, threads: int = 0):
    """d logZ / d Q (n x n float64; upper triangle incl. diagonal, zeros below)."""
    Q, isf = _prep(Q)
    if not isf:
        Q = Q.astype(np.float32)
    lib = _load()
    n = Q.shape[0]
    if logz_value is None:
        logz_value = logz(Q, beta, threads)
    G = np.empty((n, n), dtype=np.float64)
    rc = lib.qo_grad_f32(_ptr(Q, ctypes.c_float), n, n, float(beta), float(logz_value),
                         _ptr(G, ctypes.c_double), threads)
    if rc != 0:
        raise ValueError("oracle grad: bad arguments")
    return G
