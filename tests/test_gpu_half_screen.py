"""The float32 walk's half-precision block screen at the edges of its
scaling: the screen works on values scaled by a power of two that puts the
inner rows' bound R_I near 2^13, with a margin that must let through every
block the float32 screen lets through.  Each case solves with the half screen
and with the float32 screen and compares both with the oracle, bit for bit:
tiny and huge magnitudes, inner rows that are zero, negligible or dominant,
integer-valued floats with ties, and the n=40 workload."""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_19373_amd import _lib, api, inputs

pytestmark = pytest.mark.gpu


def _u64(xs):
    return [int(x) & (2**64 - 1) for x in xs]


def _both(Q, k):
    saved = _lib.get_tuning(_lib.TUNE_HALF_SCREEN)
    try:
        out = []
        for h in (1, -1):
            _lib.set_tuning(_lib.TUNE_HALF_SCREEN, h)
            e, m = api.solve(Q, k)
            out.append((e.cpu().numpy(), m.cpu().numpy()))
        return out
    finally:
        _lib.set_tuning(_lib.TUNE_HALF_SCREEN, saved)


def _check(Q, k):
    (eh, mh), (ef, mf) = _both(Q, k)
    E, M = oracle.topk(Q, k)
    assert _u64(mh) == _u64(M) and np.array_equal(eh, E)
    assert _u64(mf) == _u64(M) and np.array_equal(ef, E)


@pytest.mark.parametrize("scale", [1e-30, 1e-6, 1.0, 1e6, 1e30])
def test_magnitudes(gpu_lib, scale):
    Q = (inputs.random_f32(21, 4000).astype(np.float64) * scale).astype(np.float32)
    print(f"half screen scale={scale}", flush=True)
    _check(Q, 9)


@pytest.mark.parametrize("inner", [1e-3, 1e5])
def test_inner_rows_small_or_dominant(gpu_lib, inner):
    # rows 0..5 are the inner bits of the walk
    n = 22
    Q = inputs.random_f32(n, 4100 + int(inner > 1))
    Q[:6, :] *= np.float32(inner)
    print(f"half screen inner rows x{inner}", flush=True)
    _check(Q, 12)


def test_inner_rows_zero(gpu_lib):
    # R_I = 0: the 64 states of every block tie exactly, so the values are
    # kept integer (the exact float path resolves ties by mask)
    Q = inputs.random_i32(22, 4150, -9, 9).astype(np.float32)
    Q[:6, :] = 0
    _check(Q, 12)


def test_integer_valued_with_ties(gpu_lib):
    Q = inputs.random_i32(20, 4200, -2, 2).astype(np.float32)
    _check(Q, 40)
    _check(np.zeros((17, 17), np.float32), 25)


def test_n40_workload_same_with_either_screen(gpu_lib):
    Q, xstar = inputs.single_n40_f32_planted()
    (eh, mh), (ef, mf) = _both(Q, 16)
    assert np.array_equal(mh, mf) and np.array_equal(eh, ef)
    assert int(mh[0]) == xstar


def test_batched_and_ranges_same_with_either_screen(gpu_lib):
    Qb, ns = inputs.batched_4096(batch=64, nlo=4, nhi=24, seed=4300)
    saved = _lib.get_tuning(_lib.TUNE_HALF_SCREEN)
    try:
        res = []
        for h in (1, -1):
            _lib.set_tuning(_lib.TUNE_HALF_SCREEN, h)
            e, m = api.solve_batched(Qb, ns, 4)
            r = api.solve_range(inputs.random_f32(26, 4301), 6, 3, 2, 5)
            res.append([t.cpu() for t in (e, m, *r)])
    finally:
        _lib.set_tuning(_lib.TUNE_HALF_SCREEN, saved)
    for a, b in zip(*res):
        assert torch.equal(a, b)


def _inner_bound(Q):
    # R_I: sum of |Q| over the walk's six inner rows, both triangles
    Qs = np.triu(Q).astype(np.int64)
    Qs = Qs + np.triu(Qs, 1).T
    return int(np.abs(Qs[:6, :]).sum())


@pytest.mark.parametrize("delta", [0, 1])
def test_int16_screen_at_its_bound(gpu_lib, delta):
    # int32 Q: the int16 screen runs when R_I <= 32767, the int32 one above;
    # both must give the oracle's answer, bit for bit
    n = 20
    Q = inputs.random_i32(n, 4400, -300, 300)
    Q[0, 0] = 0
    Q[0, 0] = 32767 + delta - _inner_bound(Q)
    assert _inner_bound(Q) == 32767 + delta and abs(int(Q[0, 0])) < 2**15
    print(f"int16 screen bound R_I={_inner_bound(Q)}", flush=True)
    _check(Q, 10)


def test_int_large_inner_rows_fall_back(gpu_lib):
    Q = inputs.random_i32(21, 4500, -5000, 5000)
    assert _inner_bound(Q) > 32767
    _check(Q, 7)


def test_int_extreme_int16_values(gpu_lib):
    # inner states whose screened values reach about +-32767
    n = 18
    Q = np.zeros((n, n), np.int32)
    Q[0, 0] = -16000
    Q[1, 1] = -16000
    Q[0, 1] = -383  # C'(0b11) = -32383; R_I counts Q01 twice: 32766
    Q[6:, 6:] = np.triu(inputs.random_i32(n - 6, 4600, -40, 40))
    assert _inner_bound(Q) <= 32767
    _check(Q, 12)


def test_int_batch_mixes_both_screens(gpu_lib):
    # a batch whose instances fall on either side of the int16 bound: the two
    # kinds of rows share the table layout
    rng = np.random.default_rng(4700)
    ns = rng.integers(8, 21, 40).astype(np.int32)
    Q = np.zeros((40, 20, 20), np.int32)
    for b, n in enumerate(ns):
        hi = 30 if b % 2 == 0 else 4000
        Q[b, :n, :n] = np.triu(rng.integers(-hi, hi + 1, (n, n)))
    saved = _lib.get_tuning(_lib.TUNE_HALF_SCREEN)
    try:
        res = []
        for h in (1, -1):
            _lib.set_tuning(_lib.TUNE_HALF_SCREEN, h)
            e, m = api.solve_batched(Q, ns, 5)
            res.append((e.cpu().numpy(), m.cpu().numpy()))
    finally:
        _lib.set_tuning(_lib.TUNE_HALF_SCREEN, saved)
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    for b, n in enumerate(ns):
        E, M = oracle.topk(Q[b, :n, :n], 5)
        assert _u64(res[0][1][b]) == _u64(M) and np.array_equal(res[0][0][b], E), b


@pytest.mark.parametrize("kind", ["f64", "i64"])
def test_wide_inputs_same_with_either_screen(gpu_lib, kind):
    # float64 / int64 Q: the half screen against the float64 walk's own
    # screen, both against the oracle
    rng = np.random.default_rng(4800)
    n = 23
    if kind == "f64":
        Q = np.triu(rng.standard_normal((n, n)) / np.sqrt(n) + 1e-9 * rng.standard_normal((n, n)))
    else:
        Q = np.triu(rng.integers(-2**36, 2**36, (n, n), dtype=np.int64))
    _check(Q, 11)
