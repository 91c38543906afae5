"""The C ABI library loads and exports every symbol include/qubo_bf.h declares;
host-side argument validation answers before any HIP call (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2310_19373_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qubo_bf.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qubo_\w+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    fns = header_functions()
    for name in ("qubo_bf_solve", "qubo_bf_solve_batched", "qubo_logz_fwd", "qubo_logz_bwd",
                 "qubo_bf_workspace_size", "qubo_last_error"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in header_functions():
        assert hasattr(L, name), name
    assert set(header_functions()) == set(_lib.SIGNATURES)


def test_version_and_error_string():
    L = _lib.lib()
    assert b"gfx950" in L.qubo_version()
    assert isinstance(L.qubo_last_error(), bytes)


def test_workspace_queries_validate():
    L = _lib.lib()
    assert L.qubo_bf_workspace_size(0, 1, 0) == 0
    assert L.qubo_bf_workspace_size(64, 1, 0) == 0
    assert L.qubo_bf_workspace_size(20, 0, 0) == 0
    assert L.qubo_bf_workspace_size(20, 57, 0) == 0   # float k above 56
    assert L.qubo_bf_workspace_size(20, 64, 1) > 0    # int k up to 64
    assert L.qubo_bf_workspace_size(20, 1, 7) == 0    # bad dtype
    assert L.qubo_bf_workspace_size(40, 16, 0) > L.qubo_bf_workspace_size(20, 16, 0)
    assert L.qubo_bf_batched_workspace_size(4096, 28, 1, 0) > 0
    assert L.qubo_bf_batched_workspace_size(4096, 41, 1, 0) == 0
    # float64 (2) and int64 (3) Q: the float64 walk; k limits as float / int
    assert L.qubo_bf_workspace_size(40, 56, 2) > 0 and L.qubo_bf_workspace_size(40, 57, 2) == 0
    assert L.qubo_bf_workspace_size(40, 64, 3) > 0
    assert L.qubo_bf_batched_workspace_size(64, 30, 4, 2) > 0 and L.qubo_bf_batched_workspace_size(64, 30, 4, 3) > 0
    assert L.qubo_bf_range_workspace_size(40, 16, 2, 4) > 0 and L.qubo_bf_workspace_size(20, 1, 4) == 0


FAKE = 256  # a non-null dummy address: every case below is rejected before use


@pytest.mark.parametrize("case,code", [
    (dict(Q=None), -1), (dict(n=0), -1), (dict(n=64), -1), (dict(ldq=5), -1),
    (dict(dt=4), -1), (dict(k=0), -1), (dict(k=57), -1), (dict(dt=2, k=57), -1), (dict(status=None), -1),
    (dict(ws_bytes=16), -3),
])
def test_solve_rejects_before_any_hip_call(case, code):
    L = _lib.lib()
    a = dict(Q=FAKE, n=10, ldq=10, dt=0, k=4, en=FAKE, masks=FAKE, status=FAKE, ws=FAKE, ws_bytes=16, stream=None)
    if code != -3:
        a["ws_bytes"] = 1 << 40
    a.update(case)
    rc = L.qubo_bf_solve(a["Q"], a["n"], a["ldq"], a["dt"], a["k"], a["en"], a["masks"], a["status"], a["ws"],
                         a["ws_bytes"], a["stream"])
    assert rc == code
    assert L.qubo_last_error()


def test_batched_rejects_before_any_hip_call():
    L = _lib.lib()
    assert L.qubo_bf_solve_batched(0, FAKE, 10, FAKE, 0, 1, FAKE, FAKE, FAKE, FAKE, 1 << 40, None) == -1
    assert L.qubo_bf_solve_batched(4, FAKE, 41, FAKE, 0, 1, FAKE, FAKE, FAKE, FAKE, 1 << 40, None) == -1
    assert L.qubo_bf_solve_batched(4, FAKE, 10, None, 0, 1, FAKE, FAKE, FAKE, FAKE, 1 << 40, None) == -1
    assert L.qubo_bf_solve_batched(4, FAKE, 10, FAKE, 0, 1, FAKE, FAKE, FAKE, FAKE, 8, None) == -3


def test_tuning_knobs_roundtrip():
    L = _lib.lib()
    old = L.qubo_bf_get_tuning(_lib.TUNE_SINGLE_OUTER_BITS)
    before = L.qubo_bf_workspace_size(40, 16, 0)
    assert L.qubo_bf_set_tuning(_lib.TUNE_SINGLE_OUTER_BITS, 9) == 0
    assert L.qubo_bf_get_tuning(_lib.TUNE_SINGLE_OUTER_BITS) == 9
    assert L.qubo_bf_workspace_size(40, 16, 0) != before   # 2^9-step tables, 8x the units
    assert L.qubo_bf_set_tuning(_lib.TUNE_SINGLE_OUTER_BITS, 14) == 0
    assert L.qubo_bf_get_tuning(_lib.TUNE_SINGLE_OUTER_BITS) == 12  # clamped to the maximum
    assert L.qubo_bf_set_tuning(_lib.TUNE_SINGLE_OUTER_BITS, 0) == 0
    assert L.qubo_bf_get_tuning(_lib.TUNE_SINGLE_OUTER_BITS) == old
    assert L.qubo_bf_set_tuning(99, 1) == -1


def test_range_and_merge_argument_checks():
    L = _lib.lib()
    assert L.qubo_bf_range_workspace_size(40, 16, 0, 4) > 0
    assert L.qubo_bf_range_workspace_size(40, 16, 0, 0) == 0      # p_bits >= 1
    assert L.qubo_bf_range_workspace_size(40, 16, 0, 28) > 0      # p_bits up to n - 12
    assert L.qubo_bf_range_workspace_size(40, 16, 0, 29) == 0
    assert L.qubo_bf_range_workspace_size(63, 8, 0, 51) > 0
    assert L.qubo_bf_range_workspace_size(14, 4, 1, 3) == 0       # p_bits <= n - 12
    ws = 1 << 40
    args = lambda pb, lo, hi: (FAKE, 30, 30, 0, 4, pb, lo, hi, FAKE, FAKE, FAKE, FAKE, ws, None)
    assert L.qubo_bf_solve_range(*args(3, 2, 2)) == -1            # empty range
    assert L.qubo_bf_solve_range(*args(3, 0, 9)) == -1            # beyond 2^p_bits
    assert L.qubo_bf_solve_range(*args(3, -1, 2)) == -1
    assert L.qubo_bf_solve_range(*args(19, 0, 1)) == -1           # p_bits > n - 12
    assert L.qubo_bf_merge_topk(0, 4, FAKE, FAKE, 0, 4, FAKE, FAKE, None) == -1
    assert L.qubo_bf_merge_topk(2, 4, FAKE, FAKE, 0, 65, FAKE, FAKE, None) == -1
    assert L.qubo_bf_merge_topk(2, 4, None, FAKE, 0, 4, FAKE, FAKE, None) == -1
    assert L.qubo_logz_moments(4, None, 8, FAKE, FAKE, FAKE, FAKE, None, FAKE, FAKE, ws, None) == -1


def test_sample_argument_checks():
    L = _lib.lib()
    assert L.qubo_logz_sample_workspace_size(16, 32) > L.qubo_logz_sample_workspace_size(16, 20) > 0
    assert L.qubo_logz_sample_workspace_size(0, 8) == 0
    assert L.qubo_logz_sample_workspace_size(4, 33) == 0
    ws = 1 << 40
    args = lambda **kw: tuple(kw.get(k, d) for k, d in (
        ("batch", 4), ("Q", FAKE), ("nmax", 8), ("ns", FAKE), ("beta", FAKE), ("nsamples", 16), ("u", FAKE),
        ("masks", FAKE), ("logz", FAKE), ("status", FAKE), ("ws", FAKE), ("ws_bytes", ws), ("stream", None)))
    assert L.qubo_logz_sample(*args(nsamples=0)) == -1
    assert L.qubo_logz_sample(*args(u=None)) == -1
    assert L.qubo_logz_sample(*args(logz=None)) == -1
    assert L.qubo_logz_sample(*args(nmax=33)) == -1
    assert L.qubo_logz_sample(*args(batch=0)) == -1
    assert L.qubo_logz_sample(*args(ws_bytes=64)) == -3


def test_noalloc_scratch_covers_every_single_solve():
    # the static workspace array of qubo_bf_solve_noalloc holds the workspace
    # of every single solve at the default tuning
    L = _lib.lib()
    for dt, kmax in ((0, 56), (1, 64), (2, 56), (3, 64)):
        for n in range(1, 64):
            for k in (1, 16, kmax):
                assert 0 < L.qubo_bf_workspace_size(n, k, dt) <= _lib.NOALLOC_SCRATCH_BYTES, (dt, n, k)


@pytest.mark.parametrize("case", [dict(Q=None), dict(n=0), dict(n=64), dict(ldq=5), dict(dt=4), dict(k=0),
                                  dict(k=57), dict(status=None), dict(masks=None)])
def test_noalloc_rejects_before_any_hip_call(case):
    L = _lib.lib()
    a = dict(Q=FAKE, n=10, ldq=10, dt=0, k=4, en=FAKE, masks=FAKE, status=FAKE, stream=None)
    a.update(case)
    rc = L.qubo_bf_solve_noalloc(a["Q"], a["n"], a["ldq"], a["dt"], a["k"], a["en"], a["masks"], a["status"],
                                 a["stream"])
    assert rc == -1
    assert L.qubo_last_error()


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 16, 40, 56])
def test_default_kprime_rule(k):
    """Float Q keeps max(2k, k + 3) candidates by default (capped at 64),
    integer Q keeps k: the default workspace is the one of that explicit K'
    and smaller than the one of K' + 1."""
    L = _lib.lib()
    want = min(max(2 * k, k + 3), 64)
    for n in (20, 40):
        assert L.qubo_bf_workspace_size(n, k, 0) == L.qubo_bf_workspace_size_kp(n, k, want, 0)
        if want < 64:
            assert L.qubo_bf_workspace_size(n, k, 0) < L.qubo_bf_workspace_size_kp(n, k, want + 1, 0)
        assert L.qubo_bf_workspace_size(n, k, 1) == L.qubo_bf_workspace_size_kp(n, k, k, 1)
        assert L.qubo_bf_workspace_size(n, k, 1) < L.qubo_bf_workspace_size_kp(n, k, k + 1, 1)


def test_kprime_argument_checks():
    L = _lib.lib()
    assert L.qubo_bf_workspace_size_kp(20, 4, 0, 0) == L.qubo_bf_workspace_size(20, 4, 0)
    assert L.qubo_bf_workspace_size_kp(30, 4, 64, 0) > L.qubo_bf_workspace_size(30, 4, 0)
    assert L.qubo_bf_workspace_size_kp(20, 4, 3, 0) == 0    # kprime < k
    assert L.qubo_bf_workspace_size_kp(20, 4, 65, 0) == 0   # kprime > 64
    assert L.qubo_bf_workspace_size_kp(20, 4, 4, 1) > 0     # integer Q: kprime = k is the default
    args = lambda kp: (FAKE, 10, 10, 0, 4, kp, FAKE, FAKE, FAKE, FAKE, 1 << 40, None)
    assert L.qubo_bf_solve_kp(*args(2)) == -1
    assert L.qubo_bf_solve_kp(*args(65)) == -1
    assert b"kprime" in L.qubo_last_error()
