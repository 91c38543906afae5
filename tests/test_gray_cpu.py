"""The host Gray-code timing baseline (Algorithm 1 with the Sec. 3.1 prefix
split, float64) against the oracle: the same minimum and argmin on every
prefix split, on prefix subsets (the oracle over the same mask blocks), with
heavy integer ties (lowest mask wins) and at the paper's worked example."""
import numpy as np
import pytest

import oracle
from oracle import gray_cpu
from paper_2310_19373_amd import inputs


@pytest.mark.parametrize("n", [1, 2, 7, 13, 18])
def test_every_split_matches_oracle(n):
    Q = inputs.random_f32(n, 3000 + n)
    E, M = oracle.topk(Q, 1)
    for m in range(0, n + 1):
        e, mk = gray_cpu.minimum(Q, m)
        assert mk == int(M[0]), (n, m)
        assert abs(e - float(E[0])) <= 1e-9 * max(1.0, abs(float(E[0])))


def test_prefix_subsets_match_oracle_blocks():
    n, m = 22, 7
    Q = inputs.random_f32(n, 3100)
    s = n - m
    rng = np.random.default_rng(3101)
    pref = rng.choice(1 << m, 9, replace=False)
    e, mk = gray_cpu.minimum(Q, m, pref)
    best = None
    for p in pref:
        E, M = oracle.topk(Q, 1, lo=int(p) << s, hi=(int(p) + 1) << s)
        if best is None or (E[0], M[0]) < best:
            best = (float(E[0]), int(M[0]))
    assert mk == best[1] and abs(e - best[0]) <= 1e-9 * abs(best[0])
    assert (mk >> s) in set(int(p) for p in pref)


def test_integer_ties_go_to_the_lowest_mask():
    # integer values are exact in float64, so the walk's running value is
    # exact and ties are decided by the mask alone
    for seed in range(4):
        Qi = inputs.random_i32(16, 3200 + seed, -1, 1)
        E, M = oracle.topk(Qi, 1)
        for m in (0, 4, 9):
            e, mk = gray_cpu.minimum(Qi.astype(np.float32), m)
            assert e == float(E[0]) and mk == int(M[0]), (seed, m)
    e, mk = gray_cpu.minimum(np.zeros((12, 12), np.float32), 3)
    assert e == 0.0 and mk == 0


def test_paper_example_signed_reading():
    # the Appendix A example, signed reading: -12 at masks 239, 247, 255
    n = 8
    Q = np.zeros((n, n), np.float32)
    for i in range(n):
        for j in range(i, n):
            Q[i, j] = i - j + 2
    for m in (0, 1, 3, 8):
        assert gray_cpu.minimum(Q, m) == (-12.0, 239)


def test_invalid_arguments():
    Q = inputs.random_f32(6, 1)
    with pytest.raises(ValueError):
        gray_cpu.minimum(Q, 7)
    with pytest.raises(ValueError):
        gray_cpu.minimum(Q, 2, [4])
    with pytest.raises(ValueError):
        gray_cpu.minimum(Q, 2, [])
