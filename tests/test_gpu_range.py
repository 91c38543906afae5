"""Prefix-range solves and their merge: each range against the oracle over the
same block of masks, the merge of a partition against the full solve (bit
for bit), uneven partitions, the int path, and the n=40 workload cut into 4
ranges at full size."""
import numpy as np
import pytest

import oracle
from paper_2310_19373_amd import api, inputs

pytestmark = pytest.mark.gpu


def _u64(xs):
    return [int(x) & (2**64 - 1) for x in xs]


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("dtype", ["f32", "i32"])
def test_ranges_against_oracle_and_merge(gpu_lib, dtype):
    n, k, pb = 22, 8, 3
    Q = inputs.random_f32(n, 500) if dtype == "f32" else inputs.random_i32(n, 501, -30, 30)
    cuts = [0, 1, 2, 5, 8]  # uneven partition of the 8 prefixes
    parts = []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        print(f"range {dtype} [{lo},{hi}) of 2^{pb}", flush=True)
        e, m = api.solve_range(Q, k, pb, lo, hi)
        E, M = oracle.topk(Q, k, lo=lo << (n - pb), hi=hi << (n - pb))
        assert _u64(_np(m)) == _u64(M), (lo, hi)
        assert np.array_equal(_np(e), E), (lo, hi)
        parts.append((e, m))
    me, mm = api.merge_topk(parts, k)
    fe, fm = api.solve(Q, k)
    assert _u64(_np(mm)) == _u64(_np(fm))
    assert np.array_equal(_np(me), _np(fe))


def test_range_smaller_than_k(gpu_lib):
    n = 13  # p_bits = 1 leaves 2^12 states per range
    Q = inputs.random_i32(n, 502, -5, 5)
    e, m = api.solve_range(Q, 64, 1, 1, 2)
    E, M = oracle.topk(Q, 64, lo=1 << 12, hi=2 << 12)
    assert _u64(_np(m)) == _u64(M) and np.array_equal(_np(e), E)


def test_merge_skips_sentinels_and_keeps_order(gpu_lib):
    import torch

    e1 = torch.tensor([-3.0, 1.0, float("inf")], dtype=torch.float64, device="cuda")
    m1 = torch.tensor([5, 9, -1], dtype=torch.int64, device="cuda")
    e2 = torch.tensor([-3.0, 0.5, 2.0], dtype=torch.float64, device="cuda")
    m2 = torch.tensor([4, 7, 1], dtype=torch.int64, device="cuda")
    e, m = api.merge_topk([(e1, m1), (e2, m2)], 5)
    assert _np(e).tolist() == [-3.0, -3.0, 0.5, 1.0, 2.0]
    assert _np(m).tolist() == [4, 5, 7, 9, 1]
    e, m = api.merge_topk([(e1, m1)], 4)
    assert _np(e).tolist()[:2] == [-3.0, 1.0] and np.isinf(_np(e)[2:]).all() and (_np(m)[2:] == -1).all()


def test_n40_in_four_ranges_equals_full_solve(gpu_lib):
    Q, xstar = inputs.single_n40_f32_planted()
    parts = []
    for p in range(4):
        print(f"n40 range {p} of 4", flush=True)
        parts.append(api.solve_range(Q, 16, 2, p, p + 1))
    me, mm = api.merge_topk(parts, 16)
    fe, fm = api.solve(Q, 16)
    assert int(_np(mm)[0]) == xstar
    assert _u64(_np(mm)) == _u64(_np(fm))
    assert np.array_equal(_np(me), _np(fe))


@pytest.mark.parametrize("dtype,k,lo,hi", [("f32", 8, 1, 2), ("f32", 16, 3, 7), ("i32", 8, 9, 16),
                                          ("i32", 40, 0, 1)])
def test_seeded_ranges_against_oracle(gpu_lib, dtype, k, lo, hi):
    # n = 26: the threshold seed runs, confined to the range's first prefix
    # (k = 40, int: K' = 40 needs the two-flip neighbours of the 22 free bits)
    n, pb = 26, 4
    Q = inputs.random_f32(n, 510) if dtype == "f32" else inputs.random_i32(n, 511, -30, 30)
    print(f"seeded range {dtype} k={k} [{lo},{hi}) of 2^{pb}", flush=True)
    e, m = api.solve_range(Q, k, pb, lo, hi)
    E, M = oracle.topk(Q, k, lo=lo << (n - pb), hi=hi << (n - pb))
    assert _u64(_np(m)) == _u64(M)
    assert np.array_equal(_np(e), E)


def test_resumable_solve_checkpoints_and_resumes(gpu_lib, tmp_path):
    import torch

    n, k, pb = 26, 8, 3
    Q = inputs.random_f32(n, 520)
    ck = str(tmp_path / "state.npz")
    e, m, done, total = api.solve_resumable(Q, k, pb, ck, max_ranges=3)
    assert (done, total) == (3, 8)
    E3, M3 = oracle.topk(Q, k, lo=0, hi=3 << (n - pb))
    assert _u64(_np(m)) == _u64(M3) and np.array_equal(_np(e), E3)
    e, m, done, _ = api.solve_resumable(Q, k, pb, ck, max_ranges=2)  # resumes at piece 3
    assert done == 5
    e, m, done, _ = api.solve_resumable(Q, k, pb, ck)
    assert done == 8
    fe, fm = api.solve(Q, k)
    assert torch.equal(e, fe) and torch.equal(m, fm)
    with pytest.raises(ValueError):
        api.solve_resumable(inputs.random_f32(n, 521), k, pb, ck)  # another instance's checkpoint
