"""Property-based parity: random sizes, input types, k and integer ranges
(small ranges force heavy ties), the GPU's k best against the oracle's, bit
for bit.  Derandomised so every run draws the same cases."""
import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from paper_2310_19373_amd import _lib, api, inputs

pytestmark = pytest.mark.gpu


def _u64(xs):
    return [int(x) & (2**64 - 1) for x in xs]


def screen_eps(Q, kind):
    # the walk's error bound: float32 Q 3 * 2^-24 * R_I + 2^-36 * sum |Q| (R_I:
    # sum |Q| over the six inner rows), float64 Q 2^-36 * sum |Q|
    A = np.abs(np.triu(Q).astype(np.float64))
    sa = A.sum()
    if kind == "f64":
        return 2.0**-36 * sa
    return 3 * 2.0**-24 * A[:6].sum() + 2.0**-36 * sa


def near_tie_within_eps(Q, k, kind):
    n = Q.shape[0]
    if 2**n < 64:
        return False  # fewer states than candidates: nothing is discarded
    E, _ = oracle.topk(Q, 64)
    return bool(E[63] - E[k - 1] <= 2 * screen_eps(Q, kind) * (1 + 1e-9))


@settings(max_examples=48, deadline=None, derandomize=True)
@given(n=st.integers(1, 24), kind=st.sampled_from(["f32", "i32", "f64", "i64"]), k=st.integers(1, 56),
       spread=st.sampled_from([1, 3, 100]), seed=st.integers(0, 2**20))
def test_random_instances_match_oracle(gpu_lib, n, kind, k, spread, seed):
    if kind == "f32":
        Q = inputs.random_f32(n, seed, scale=float(spread) / 10)
    elif kind == "f64":
        Q = inputs.random_f32(n, seed).astype(np.float64) * (spread / 7.0)
    else:
        Q = inputs.random_i32(n, seed, -spread, spread)
        if kind == "i64":
            Q = Q.astype(np.int64) * (2**30 + 7)  # sums beyond the int32 walk's 2^28
    print(f"property n={n} {kind} k={k} spread={spread} seed={seed}", flush=True)
    try:
        e, m = api.solve(Q, k)
    except api.UncertainError:
        # allowed only for float data whose 64 best states (the list length of
        # the retry) hold a real near-tie: the certificate needs the 64th
        # candidate key, minus the screen's error bound eps, above the k-th
        # rescored energy, and a key is within eps of its state's exact value
        assert kind in ("f32", "f64")
        assert near_tie_within_eps(Q, k, kind), "certificate failed without a near-tie in the oracle's top 64"
        return
    E, M = oracle.topk(Q, k)
    assert _u64(m.cpu().numpy()) == _u64(M)
    assert np.array_equal(e.cpu().numpy(), E)
