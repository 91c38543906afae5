"""Pins for the CPU oracle: checks against what the paper and the mathematics
fix, never against the oracle itself.

Each test names the passage it follows.  Independent evaluators written here
(pure-Python pair sums, numpy's x @ Q @ x of the naive solver in Sec. 3, a
Python Gray-code walk of Algorithm 1) are separate code from the oracle's C.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2310_19373_amd import inputs


# ---------------------------------------------------------------- helpers

def py_energy(Q, mask):
    """Eq. 1 as a pair sum over i <= j, pure Python (float or int)."""
    n = Q.shape[0]
    x = [(mask >> i) & 1 for i in range(n)]
    tot = 0 if Q.dtype.kind == "i" else 0.0
    for i in range(n):
        for j in range(i, n):
            if x[i] and x[j]:
                tot += Q[i, j].item()
    return tot


def all_bits(n):
    m = np.arange(1 << n, dtype=np.int64)
    return ((m[:, None] >> np.arange(n)) & 1).astype(np.float64)


def naive_numpy_energies(Q):
    """The naive solver's x @ Q @ x (Sec. 3) for every x, float64."""
    n = Q.shape[0]
    X = all_bits(n)
    Qf = np.triu(Q.astype(np.float64))
    return np.einsum("bi,ij,bj->b", X, Qf, X)


def brute_topk(vals, k):
    """k lowest (value, index) pairs, ties to the lower index."""
    order = sorted(range(len(vals)), key=lambda i: (vals[i], i))[:k]
    return [vals[i] for i in order], order


def local_field(Q, x):
    """h_l(x) = Q_ll + sum_{j != l} S_lj x_j, S = triu(Q,1) + triu(Q,1)^T (the bracket of Eq. 2)."""
    off = np.triu(Q, 1)
    S = off + off.T
    return np.diag(Q) + S @ x


# ----------------------------------------------------------- energy pins

@pytest.mark.parametrize("dtype", ["f32", "i32"])
def test_zero_vector_has_value_zero(dtype):
    # Sec. 2.1: f(0) = 0 for every Q.
    for seed in range(5):
        Q = inputs.random_f32(13, seed) if dtype == "f32" else inputs.random_i32(13, seed)
        assert oracle.energy(Q, 0) == 0


def test_energy_equals_pair_sum_int():
    # Eq. 1 summed pair by pair; integers are exact in any order.
    Q = inputs.random_i32(9, 11)
    E = oracle.energies(Q, np.arange(1 << 9, dtype=np.uint64))
    assert all(int(E[m]) == py_energy(Q, m) for m in range(1 << 9))


def test_energy_equals_pair_sum_float():
    Q = inputs.random_f32(9, 12)
    E = oracle.energies(Q, np.arange(1 << 9, dtype=np.uint64))
    ref = [py_energy(Q, m) for m in range(1 << 9)]
    np.testing.assert_allclose(E, ref, rtol=0, atol=1e-12)


def test_energy_equals_naive_xQx():
    # Sec. 3: the naive solver evaluates v = x @ Q @ x.
    Q = inputs.random_f32(12, 13)
    E = oracle.energies(Q, np.arange(1 << 12, dtype=np.uint64))
    np.testing.assert_allclose(E, naive_numpy_energies(Q), rtol=0, atol=1e-11)


def test_lower_triangle_is_ignored():
    # Eq. 1 sums over i <= j only; Q is upper triangular.
    Q = inputs.random_i32(10, 14)
    Qg = Q.copy()
    Qg[np.tril_indices(10, -1)] = 77
    masks = np.arange(1 << 10, dtype=np.uint64)
    assert np.array_equal(oracle.energies(Q, masks), oracle.energies(Qg, masks))


def test_delta_rule_eq2():
    # Eq. 2: flipping bit l changes f by s_l * (column-l sum + Q_ll + row-l sum),
    # s_l = new - old bit; here via h_l(x).  Exact in integers for every x, l.
    n = 9
    Q = inputs.random_i32(n, 15)
    E = oracle.energies(Q, np.arange(1 << n, dtype=np.uint64))
    for m in range(1 << n):
        x = np.array([(m >> i) & 1 for i in range(n)], dtype=np.int64)
        h = local_field(Q.astype(np.int64), x)
        for l in range(n):
            s = 1 - 2 * x[l]
            assert E[m ^ (1 << l)] - E[m] == s * h[l]


def test_half_field_invariant():
    # f(x) = 1/2 sum_i x_i (Q_ii + h_i(x)) (each pair counted from both ends).
    n = 8
    Q = inputs.random_i32(n, 16)
    E = oracle.energies(Q, np.arange(1 << n, dtype=np.uint64))
    for m in range(1 << n):
        x = np.array([(m >> i) & 1 for i in range(n)], dtype=np.int64)
        h = local_field(Q.astype(np.int64), x)
        assert 2 * E[m] == int((x * (np.diag(Q) + h)).sum())


# ------------------------------------------------------------ top-k pins

@pytest.mark.parametrize("n,k", [(1, 1), (1, 2), (2, 4), (5, 3), (7, 1), (8, 256), (10, 3)])
def test_topk_int_equals_bruteforce(n, k):
    Q = inputs.random_i32(n, 100 + n)
    vals = [py_energy(Q, m) for m in range(1 << n)]
    E, M = oracle.topk(Q, k)
    bv, bi = brute_topk(vals, k)
    kk = min(k, 1 << n)
    assert list(E[:kk]) == bv and list(M[:kk]) == bi
    assert all(E[kk:] == np.iinfo(np.int64).max) and all(M[kk:] == np.uint64(2**64 - 1))


@pytest.mark.parametrize("n,k", [(3, 2), (9, 5), (14, 8), (16, 16)])
def test_topk_float_equals_naive(n, k):
    Q = inputs.random_f32(n, 200 + n)
    vals = naive_numpy_energies(Q)
    E, M = oracle.topk(Q, k)
    order = np.lexsort((np.arange(len(vals)), vals))[:k]
    assert list(M) == list(order)
    np.testing.assert_allclose(E, vals[order], rtol=0, atol=1e-11)


def test_ties_go_to_lowest_natural_mask():
    # Zero Q: every state ties at 0, so the k best are masks 0..k-1.
    Q = np.zeros((6, 6), dtype=np.int32)
    E, M = oracle.topk(Q, 10)
    assert list(E) == [0] * 10 and list(M) == list(range(10))
    Qf = np.zeros((6, 6), dtype=np.float32)
    E, M = oracle.topk(Qf, 5)
    assert list(E) == [0.0] * 5 and list(M) == list(range(5))


def test_diagonal_closed_form():
    # Diagonal Q: f(x) = sum_i Q_ii x_i, minimum sum_i min(0, Q_ii) at the mask of
    # the negative entries (zero entries stay 0: lowest mask).
    rng = np.random.default_rng(5)
    for n in (4, 9, 13):
        d = rng.integers(-9, 10, n).astype(np.int32)
        d[0] = 0
        Q = np.diag(d).astype(np.int32)
        E, M = oracle.topk(Q, 1)
        assert E[0] == np.minimum(d, 0).sum()
        assert M[0] == sum(1 << i for i in range(n) if d[i] < 0)


def test_positive_and_minus_identity():
    n = 9
    rng = np.random.default_rng(6)
    Q = np.triu(rng.integers(1, 50, (n, n))).astype(np.int32)
    E, M = oracle.topk(Q, 2)
    assert (E[0], M[0]) == (0, 0)
    i = int(np.argmin(np.diag(Q)))
    assert (E[1], M[1]) == (int(np.diag(Q).min()), 1 << i)
    E, M = oracle.topk(-np.eye(n, dtype=np.int32), 1)
    assert (E[0], M[0]) == (-n, (1 << n) - 1)


def test_complement_symmetry():
    # f_Q(1 - x) = f_Q(1) + f_Qt(x), Qt_ij = Q_ij (i < j), Qt_ii = -Q_ii - sum_{j != i} S_ij.
    n = 8
    Q = inputs.random_i32(n, 17).astype(np.int64)
    off = np.triu(Q, 1)
    S = off + off.T
    Qt = off.copy()
    Qt[np.arange(n), np.arange(n)] = -np.diag(Q) - S.sum(axis=1)
    full = (1 << n) - 1
    masks = np.arange(1 << n, dtype=np.uint64)
    EQ = oracle.energies(Q.astype(np.int32), masks)
    Et = oracle.energies(Qt.astype(np.int32), masks)
    for m in range(1 << n):
        assert EQ[full ^ m] == EQ[full] + Et[m]


def _c_main_q(literal: bool):
    # Appendix A example: n = 8, qubo[i][j] = (double)(i - j + 2) for i <= j, with
    # i, j of type size_t.  Signed reading: the intended small integers; literal
    # reading: i - j + 2 wraps modulo 2^64 when j > i + 2.
    n = 8
    Q = np.zeros((n, n), dtype=np.float64)
    for i in range(n):
        for j in range(i, n):
            v = i - j + 2
            Q[i, j] = float(v % (1 << 64)) if literal else float(v)
    return Q


def test_c_main_example_signed_reading():
    Q = _c_main_q(False).astype(np.int32)
    vals = [py_energy(Q, m) for m in range(256)]
    E, M = oracle.topk(Q, 5)
    bv, bi = brute_topk(vals, 5)
    assert list(E) == bv and list(M) == bi
    # three states tie at the minimum; the lowest natural mask wins
    assert list(E[:3]) == [-12] * 3 and list(M[:3]) == [239, 247, 255]
    assert (E[3], M[3]) == (-11, 231) and (E[4], M[4]) == (-10, 215)


def test_c_main_example_literal_reading():
    Q = _c_main_q(True).astype(np.float32)
    E, M = oracle.topk(Q, 1)
    assert E[0] == 0.0 and M[0] == 0


@pytest.mark.parametrize("threads", [1, 2, 7])
def test_thread_count_invariance(threads):
    Q = inputs.random_f32(15, 18)
    E1, M1 = oracle.topk(Q, 9, threads=1)
    Et, Mt = oracle.topk(Q, 9, threads=threads)
    assert np.array_equal(E1, Et) and np.array_equal(M1, Mt)


@pytest.mark.parametrize("m", [0, 1, 3, 11])
def test_prefix_split_min_of_minima(m):
    # Sec. 3.1 / Fig. 3: fixing the last m bits gives 2^m sub-problems whose
    # minima, min-combined, give the global minimum.
    n = 12
    Q = inputs.random_f32(n, 19)
    E, M = oracle.topk(Q, 1)
    sub = [oracle.topk(Q, 1, lo=p << (n - m), hi=(p + 1) << (n - m)) for p in range(1 << m)]
    best = min(sub, key=lambda r: (r[0][0], r[1][0]))
    assert best[0][0] == E[0] and best[1][0] == M[0]


def gray_walk_min(Q):
    """Algorithm 1 in plain Python: flip bit CTZ(i), update v by Eq. 2 (strict <).

    Starts from x = 0 with v = v* = 0 (the code's initialisation, Sec. 3)."""
    n = Q.shape[0]
    x = [0] * n
    v = 0.0
    best_v, best_x = 0.0, 0
    for i in range(1, 1 << n):
        l = (i & -i).bit_length() - 1
        x[l] = 1 - x[l]
        d = sum(Q[a, l] * x[a] for a in range(l)) + Q[l, l] + sum(Q[l, b] * x[b] for b in range(l + 1, n))
        v += (2 * x[l] - 1) * d
        if v < best_v:
            best_v = v
            best_x = sum(x[a] << a for a in range(n))
    return best_v, best_x


def test_flip_sequence_is_binary_carry_sequence():
    # Sec. 2.2: the flip indices 0,1,0,2,0,1,0,3,0,1,0,2,0 are CTZ(1..13), and
    # consecutive reflected Gray codes g(t) = t ^ (t >> 1) differ in that bit.
    printed = [0, 1, 0, 2, 0, 1, 0, 3, 0, 1, 0, 2, 0]
    ctz = [(t & -t).bit_length() - 1 for t in range(1, 14)]
    assert ctz == printed
    for t in range(1, 1 << 12):
        assert (t ^ (t >> 1)) ^ ((t - 1) ^ ((t - 1) >> 1)) == 1 << ((t & -t).bit_length() - 1)
    assert sorted(t ^ (t >> 1) for t in range(1 << 12)) == list(range(1 << 12))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_algorithm1_gray_walk_agrees(seed):
    # Algorithm 1 reaches the same minimum value as the oracle; with no float
    # ties, the same minimiser.
    Q = inputs.random_i32(10, 300 + seed)
    v, xm = gray_walk_min(Q.astype(np.int64))
    E, M = oracle.topk(Q, 1)
    assert v == E[0]
    assert oracle.energy(Q, xm) == E[0]


@pytest.mark.parametrize("seed", range(8))
def test_planted_minimiser_is_unique_argmin(seed):
    # The planted construction (diagonal shift) makes x* the unique minimiser
    # with margin >= 1.
    Q, xstar = inputs.planted_f32(12, 1000 + seed)
    E, M = oracle.topk(Q, 2)
    assert M[0] == xstar
    assert E[1] - E[0] >= 1.0


def test_planted_n40_generator_claims():
    Q, xstar = inputs.single_n40_f32_planted()
    assert Q.dtype == np.float32 and Q.shape == (40, 40)
    assert not np.any(np.tril(Q, -1))
    assert bin(xstar).count("1") == 20


def test_config1_against_numpy_bruteforce():
    # n=20 float32 N(0,1), seed 0: an independent vectorised brute force.
    Q = inputs.single_n20_f32()
    n = 20
    Qf = np.triu(Q.astype(np.float64))
    vals = np.empty(1 << n)
    step = 1 << 16
    for a in range(0, 1 << n, step):
        m = np.arange(a, a + step, dtype=np.int64)
        X = ((m[:, None] >> np.arange(n)) & 1).astype(np.float64)
        vals[a:a + step] = np.einsum("bi,ij,bj->b", X, Qf, X)
    order = np.lexsort((np.arange(1 << n), vals))[:8]
    E, M = oracle.topk(Q, 8)
    assert list(M) == list(order)
    np.testing.assert_allclose(E, vals[order], rtol=0, atol=1e-10)


# ------------------------------------------------------- log-partition pins

def brute_logz(Q, beta):
    a = -beta * naive_numpy_energies(Q)
    mx = a.max()
    return mx + math.log(np.exp(a - mx).sum())


@pytest.mark.parametrize("beta", [0.5, 1.0, 4.0, -0.7])
def test_logz_against_bruteforce(beta):
    Q = inputs.random_f32(12, 21, scale=1 / math.sqrt(12))
    assert abs(oracle.logz(Q, beta) - brute_logz(Q, beta)) < 1e-11


def test_logz_closed_forms():
    n = 10
    Z = np.zeros((n, n), dtype=np.float32)
    assert abs(oracle.logz(Z, 1.3) - n * math.log(2)) < 1e-12
    d = np.random.default_rng(7).normal(0, 1, n).astype(np.float32)
    D = np.diag(d).astype(np.float32)
    beta = 1.7
    ref = sum(math.log1p(math.exp(-beta * float(v))) for v in d)
    assert abs(oracle.logz(D, beta) - ref) < 1e-12
    # beta = 0 counts the states
    Q = inputs.random_f32(n, 22)
    assert abs(oracle.logz(Q, 0.0) - n * math.log(2)) < 1e-12


def test_logz_beta_derivative_and_convexity():
    # d logZ / d beta = -E_p[f]; logZ is convex in beta.
    Q = inputs.random_f32(11, 23, scale=1 / math.sqrt(11))
    b, h = 1.3, 1e-4
    lz, mean = oracle.logz(Q, b, with_mean=True)
    fd = (oracle.logz(Q, b + h) - oracle.logz(Q, b - h)) / (2 * h)
    assert abs(fd + mean) < 1e-7
    assert oracle.logz(Q, b + h) + oracle.logz(Q, b - h) - 2 * lz > 0


def test_logz_large_beta_limit():
    # For large beta, logZ ~ -beta E_min + log(multiplicity of the minimum).
    Q = np.triu(np.random.default_rng(8).integers(-5, 6, (9, 9))).astype(np.float32)
    E, M = oracle.topk(Q.astype(np.int32), 512)
    mult = int((E == E[0]).sum())
    beta = 60.0
    assert abs(oracle.logz(Q, beta) - (-beta * E[0] + math.log(mult))) < 1e-12


# -------------------------------------------------------------- gradient pins

def brute_grad(Q, beta):
    n = Q.shape[0]
    X = all_bits(n)
    e = naive_numpy_energies(Q)
    a = -beta * e
    p = np.exp(a - a.max())
    p /= p.sum()
    M = np.einsum("b,bi,bj->ij", p, X, X)
    return -beta * np.triu(M)


def test_grad_against_bruteforce_moments():
    Q = inputs.random_f32(10, 24, scale=1 / math.sqrt(10))
    for beta in (0.5, 4.0):
        G = oracle.grad(Q, beta)
        np.testing.assert_allclose(G, brute_grad(Q, beta), rtol=0, atol=1e-13)


def test_grad_closed_forms():
    n = 7
    beta = 0.9
    G = oracle.grad(np.zeros((n, n), dtype=np.float32), beta)
    iu = np.triu_indices(n, 1)
    np.testing.assert_allclose(np.diag(G), -beta / 2, atol=1e-14)
    np.testing.assert_allclose(G[iu], -beta / 4, atol=1e-14)
    assert np.all(np.tril(G, -1) == 0)
    d = np.random.default_rng(9).normal(0, 1, n).astype(np.float32)
    G = oracle.grad(np.diag(d).astype(np.float32), beta)
    sig = 1.0 / (1.0 + np.exp(beta * d.astype(np.float64)))
    np.testing.assert_allclose(np.diag(G), -beta * sig, atol=1e-14)
    np.testing.assert_allclose(G[iu], (-beta * np.outer(sig, sig))[iu], atol=1e-14)


def test_grad_moment_bounds():
    Q = inputs.random_f32(9, 25)
    beta = 1.0
    Mo = oracle.grad(Q, beta) / -beta
    m1 = np.diag(Mo)
    iu = np.triu_indices(9, 1)
    assert np.all(Mo[iu] >= -1e-15)
    assert np.all(Mo[iu] <= np.minimum.outer(m1, m1)[iu] + 1e-15)


def test_grad_central_finite_differences_and_richardson():
    # Central differences of logZ in float64, h = 1e-3; halving h cuts the error ~4x.
    n = 8
    Q = inputs.random_f32(n, 26, scale=1 / math.sqrt(n))
    beta = 1.0
    G = oracle.grad(Q, beta)
    Qd = Q.astype(np.float64)

    def lz(Qm):
        # logZ of a float64 matrix through the brute-force evaluator
        X = all_bits(n)
        a = -beta * np.einsum("bi,ij,bj->b", X, np.triu(Qm), X)
        mx = a.max()
        return mx + math.log(np.exp(a - mx).sum())

    errs = {}
    for h in (1e-3, 5e-4):
        e = 0.0
        for i in range(n):
            for j in range(i, n):
                P = Qd.copy()
                P[i, j] += h
                Mi = Qd.copy()
                Mi[i, j] -= h
                fd = (lz(P) - lz(Mi)) / (2 * h)
                e = max(e, abs(fd - G[i, j]))
        errs[h] = e
    assert errs[1e-3] < 1e-5
    assert errs[5e-4] < errs[1e-3] / 2.5


# ------------------------------------------------ float64 and int64 inputs

def _fraction_energy(Q, mask):
    """Eq. 1 in exact rational arithmetic over the stored float64 values."""
    from fractions import Fraction

    n = Q.shape[0]
    x = [(mask >> i) & 1 for i in range(n)]
    return sum((Fraction(float(Q[i, j])) for i in range(n) for j in range(i, n) if x[i] and x[j]), Fraction(0))


def test_f64_energy_within_rounding_of_exact_sum():
    # Eq. 1 on float64 Q: the oracle's float64 sum lies within n^2 roundings of
    # the exact rational value; values are not float32-representable
    rng = np.random.default_rng(71)
    n = 9
    Q = np.triu(rng.standard_normal((n, n)) * 1e3 + 1e-7)
    tol = n * n * 2.0**-53 * float(np.abs(Q).sum())
    E = oracle.energies(Q, np.arange(1 << n, dtype=np.uint64))
    for mask in range(1 << n):
        assert abs(E[mask] - float(_fraction_energy(Q, mask))) <= tol
    assert E[0] == 0.0


def test_f64_reduces_to_f32_on_float32_values():
    # float32 values widened to float64 are the same numbers: both input types
    # give bitwise the same energies and the same selection
    Q32 = inputs.random_f32(12, 72)
    Q64 = Q32.astype(np.float64)
    masks = np.arange(1 << 12, dtype=np.uint64)
    assert np.array_equal(oracle.energies(Q64, masks), oracle.energies(Q32, masks))
    e32, m32 = oracle.topk(Q32, 9)
    e64, m64 = oracle.topk(Q64, 9)
    assert np.array_equal(e32, e64) and np.array_equal(m32, m64)


@pytest.mark.parametrize("n,k", [(1, 2), (5, 32), (6, 5), (10, 12)])
def test_topk_f64_and_i64_equal_bruteforce(n, k):
    # Sec. 3 naive enumeration with Python's exact integers (values far beyond
    # int32) and exact rationals: the k smallest by (energy, mask)
    rng = np.random.default_rng(73 + n)
    Qi = np.triu(rng.integers(-2**40, 2**40, (n, n), dtype=np.int64))
    vals = [py_energy(Qi, m) for m in range(1 << n)]
    E, M = oracle.topk(Qi, k)
    ref = sorted((v, m) for m, v in enumerate(vals))[:k]
    assert [int(e) for e in E[:len(ref)]] == [v for v, _ in ref]
    assert [int(m) for m in M[:len(ref)]] == [m for _, m in ref]
    Qf = np.triu(rng.standard_normal((n, n)) * 7.3)
    exact = [_fraction_energy(Qf, m) for m in range(1 << n)]
    E, M = oracle.topk(Qf, k)
    ref = sorted((v, m) for m, v in enumerate(exact))[:k]
    assert [int(m) for m in M[:len(ref)]] == [m for _, m in ref]
    assert all(abs(e - float(v)) <= 1e-12 * max(1.0, abs(float(v))) for e, (v, _) in zip(E, ref))
    if k > 1 << n:
        assert np.isinf(E[1 << n:]).all()


def test_i64_matches_i32_on_int32_values_and_diagonal_closed_form():
    Q32 = inputs.random_i32(11, 74)
    e32, m32 = oracle.topk(Q32, 7)
    e64, m64 = oracle.topk(Q32.astype(np.int64), 7)
    assert np.array_equal(e32, e64) and np.array_equal(m32, m64)
    # diagonal Q: the minimum is the sum of the negative diagonal entries, at the
    # mask of those entries (zeros stay 0)
    d = np.array([5 * 2**40, -3 * 2**41, 0, -7, 2**45, -1], dtype=np.int64)
    E, M = oracle.topk(np.diag(d), 1)
    assert int(E[0]) == int(d[d < 0].sum())
    assert int(M[0]) == sum(1 << i for i in range(d.size) if d[i] < 0)
