"""Parity at the sizes where the bit split changes, beyond what a full oracle
run reaches, and at n > 40.

* Plan sweep: every n in 27..44, float32 and int32 Q, three random prefix
  ranges of 2^22 or 2^23 masks (the fixed-prefix sub-walks of Sec. 3.1), each
  compared bit for bit with the oracle's top-k over the same block of masks.
* Sampled prefixes at n = 40: 64 random prefixes of 2^22 masks of the planted
  n=40 workload; the GPU's and the oracle's top-k of each block must be equal
  (both directions: the same set, in the same order, with the same values).
* Planted minimisers: full solves at n in {33, 36, 39, 41, 44} and, at n = 48
  and 63, the range of 2^24 masks that holds x*: x* comes first with the
  oracle's energy and, where the oracle can run the range, the whole top-k
  equals the oracle's.
* int64 and float64 Q at n = 63: a range of 2^20 masks against the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2310_19373_amd import api, inputs

pytestmark = pytest.mark.gpu


def _u64(xs):
    return [int(x) & (2**64 - 1) for x in xs]


def _np(t):
    return t.cpu().numpy()


def _sweep_instance(n, kind):
    if kind == "f32":
        return inputs.random_f32(n, 4000 + n, scale=1 / np.sqrt(n))
    return inputs.random_i32(n, 4100 + n)


@pytest.mark.parametrize("n", list(range(27, 45)))
@pytest.mark.parametrize("kind", ["f32", "i32"])
def test_plan_sweep_prefix_ranges_against_oracle(gpu_lib, n, kind):
    Q = _sweep_instance(n, kind)
    rng = np.random.default_rng(4200 + n + (0 if kind == "f32" else 100))
    k = 8
    for span_bits in (22, 22, 23):
        p_bits = n - span_bits
        p = int(rng.integers(0, 1 << p_bits))
        lo, hi = p << span_bits, (p + 1) << span_bits
        print(f"sweep {kind} n={n} p_bits={p_bits} prefix={p}", flush=True)
        e, m = api.solve_range(Q, k, p_bits, p, p + 1)
        E, M = oracle.topk(Q, k, lo=lo, hi=hi)
        assert _u64(_np(m)) == _u64(M), (n, kind, p_bits, p)
        assert np.array_equal(_np(e), E), (n, kind, p_bits, p)


def test_n40_sampled_prefixes_both_ways(gpu_lib):
    Q, _ = inputs.single_n40_f32_planted()
    rng = np.random.default_rng(4040)
    p_bits, k = 18, 16
    prefixes = sorted(int(p) for p in rng.choice(1 << p_bits, 64, replace=False))
    for p in prefixes:
        lo, hi = p << 22, (p + 1) << 22
        print(f"n40 prefix {p}", flush=True)
        e, m = api.solve_range(Q, k, p_bits, p, p + 1)
        E, M = oracle.topk(Q, k, lo=lo, hi=hi)
        g_m, g_e = _u64(_np(m)), _np(e)
        # GPU -> oracle: every returned state lies in the block, has the
        # oracle's value and is among the oracle's k best
        assert all(lo <= x < hi for x in g_m), p
        assert np.array_equal(oracle.energies(Q, np.array(g_m, dtype=np.uint64)), g_e), p
        # oracle -> GPU: the oracle's k best are exactly the returned ones, in order
        assert g_m == _u64(M), p
        assert np.array_equal(g_e, E), p


@pytest.mark.parametrize("n", [33, 36, 39, 41, 44])
def test_planted_full_solves(gpu_lib, n):
    Q, xstar = inputs.planted_f32(n, 4300 + n)
    k = 16
    print(f"planted n={n}", flush=True)
    e, m = api.solve(Q, k)
    g_m, g_e = _u64(_np(m)), _np(e)
    assert g_m[0] == xstar
    assert g_e[0] == oracle.energy(Q, xstar)
    # x* is the unique minimum by at least 1 (the planting margin)
    assert g_e[1] >= g_e[0] + 1.0
    # every returned energy is the oracle's value of its mask; ascending by
    # (energy, mask), distinct masks
    assert np.array_equal(oracle.energies(Q, np.array(g_m, dtype=np.uint64)), g_e)
    assert len(set(g_m)) == k
    assert all((g_e[i], g_m[i]) < (g_e[i + 1], g_m[i + 1]) for i in range(k - 1))


@pytest.mark.parametrize("n", [48, 63])
def test_planted_beyond_40_by_the_range_holding_xstar(gpu_lib, n):
    Q, xstar = inputs.planted_f32(n, 4400 + n)
    k, span = 8, 24
    p_bits = n - span
    p = xstar >> span
    lo, hi = p << span, (p + 1) << span
    print(f"planted n={n} range of prefix {p} (p_bits={p_bits})", flush=True)
    e, m = api.solve_range(Q, k, p_bits, p, p + 1)
    g_m, g_e = _u64(_np(m)), _np(e)
    assert g_m[0] == xstar
    assert g_e[0] == oracle.energy(Q, xstar)
    E, M = oracle.topk(Q, k, lo=lo, hi=hi)
    assert g_m == _u64(M)
    assert np.array_equal(g_e, E)
    # a neighbouring prefix: no x*, still the oracle's top-k of its block
    q = p ^ 1
    e2, m2 = api.solve_range(Q, k, p_bits, q, q + 1)
    E2, M2 = oracle.topk(Q, k, lo=q << span, hi=(q + 1) << span)
    assert _u64(_np(m2)) == _u64(M2) and np.array_equal(_np(e2), E2)


@pytest.mark.parametrize("dtype", [np.int64, np.float64])
def test_wide_dtypes_at_n63_range_against_oracle(gpu_lib, dtype):
    """int64 and float64 Q at n = 63, the widest mask: one prefix range of 2^20
    masks, bit for bit against the oracle's top-k of the same block.  The merge
    and rescoring launch then holds the largest n x n block of 8-byte Q."""
    n, span, k = 63, 20, 16
    rng = np.random.default_rng(6363 if dtype is np.int64 else 6364)
    if dtype is np.int64:
        Q = np.triu(rng.integers(-1000, 1001, (n, n))).astype(np.int64)
    else:
        Q = np.triu(rng.standard_normal((n, n)) / np.sqrt(n)).astype(np.float64)
    p_bits = n - span
    p = int(rng.integers(0, 1 << p_bits))
    print(f"n=63 {np.dtype(dtype).name} range of prefix {p} (p_bits={p_bits})", flush=True)
    e, m = api.solve_range(Q, k, p_bits, p, p + 1)
    E, M = oracle.topk(Q, k, lo=p << span, hi=(p + 1) << span)
    assert _u64(_np(m)) == _u64(M)
    assert np.array_equal(_np(e), E)
