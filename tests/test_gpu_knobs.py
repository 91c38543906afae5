"""Speed-only tuning knobs leave every output bit-identical.

Work distribution (dynamic XCD-segmented queue vs static round-robin, chunk
caps), the threshold seed (on, off, more descents), the launch shape
(outer bits, waves per CU) and the float32 walk's block screen (packed float16
or float32) change which wave walks which states and when, never the results.  Each case compares against the default setting and, on
small sizes, against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_19373_amd import _lib, api, autotune, inputs

pytestmark = pytest.mark.gpu

SETTINGS = [
    {},
    {"dyn": -1},
    {"dyn": -1, "chunk_single": 1, "chunk_batched": 1},
    {"seed": -1},
    {"seed": 16},
    {"chunk_single": 16, "chunk_batched": 32},
    {"waves_per_cu": 4},
    {"single_outer": 8, "batched_outer": 6},
    {"half": -1},
]
KNOB = {"dyn": _lib.TUNE_DYNAMIC_QUEUE, "seed": _lib.TUNE_SEED_SWEEPS, "chunk_single": _lib.TUNE_CHUNK_SINGLE,
        "chunk_batched": _lib.TUNE_CHUNK_BATCHED, "waves_per_cu": _lib.TUNE_WAVES_PER_CU,
        "single_outer": _lib.TUNE_SINGLE_OUTER_BITS, "batched_outer": _lib.TUNE_BATCHED_OUTER_BITS,
        "half": _lib.TUNE_HALF_SCREEN}


class _knobs:
    def __init__(self, setting):
        self.setting = setting

    def __enter__(self):
        self.saved = {k: _lib.get_tuning(KNOB[k]) for k in KNOB}
        for k, v in self.setting.items():
            _lib.set_tuning(KNOB[k], v)

    def __exit__(self, *exc):
        for k, v in self.saved.items():
            _lib.set_tuning(KNOB[k], v)


def _u64(xs):
    return [int(x) & (2**64 - 1) for x in xs]


def _batch(seed, batch, lo, hi, dtype):
    rng = np.random.default_rng(seed)
    ns = rng.integers(lo, hi + 1, batch).astype(np.int32)
    q = np.zeros((batch, hi, hi), dtype=np.float32 if dtype == "f32" else np.int32)
    for b, n in enumerate(ns):
        if dtype == "f32":
            q[b, :n, :n] = np.triu(rng.standard_normal((n, n))).astype(np.float32)
        else:
            q[b, :n, :n] = np.triu(rng.integers(-50, 51, (n, n)))
    return q, ns


@pytest.fixture(scope="module")
def cases():
    qf = inputs.random_f32(27, 71)
    qi = inputs.random_i32(26, 72)
    bf, nsf = _batch(73, 300, 1, 22, "f32")
    bi, nsi = _batch(74, 5, 3, 9, "i32")  # fewer work units than queue segments
    out = {}
    with _knobs({}):
        out["single_f32"] = [t.cpu() for t in api.solve(qf, k=12)]
        out["single_i32"] = [t.cpu() for t in api.solve(qi, k=7)]
        out["batched_f32"] = [t.cpu() for t in api.solve_batched(bf, nsf, k=3)]
        out["batched_i32"] = [t.cpu() for t in api.solve_batched(bi, nsi, k=64)]
    return (qf, qi, bf, nsf, bi, nsi), out


def test_defaults_against_oracle(gpu_lib, cases):
    (qf, qi, bf, nsf, bi, nsi), ref = cases
    oe, om = oracle.topk(qf, 12)
    assert _u64(ref["single_f32"][1]) == _u64(om)
    oe, om = oracle.topk(qi, 7)
    assert [int(e) for e in ref["single_i32"][0]] == [int(e) for e in oe]
    for b in range(0, len(nsf), 13):
        n = int(nsf[b])
        oe, om = oracle.topk(np.ascontiguousarray(bf[b, :n, :n]), 3)
        assert _u64(ref["batched_f32"][1][b]) == _u64(om), b
    for b in range(len(nsi)):
        n = int(nsi[b])
        oe, om = oracle.topk(np.ascontiguousarray(bi[b, :n, :n]), 64)
        assert [int(e) for e in ref["batched_i32"][0][b]] == [int(e) for e in oe], b
        assert _u64(ref["batched_i32"][1][b]) == _u64(om), b


@pytest.mark.parametrize("setting", SETTINGS[1:], ids=lambda s: ",".join(f"{k}={v}" for k, v in s.items()))
def test_setting_is_bit_identical(gpu_lib, cases, setting):
    (qf, qi, bf, nsf, bi, nsi), ref = cases
    print("knobs", setting, flush=True)
    with _knobs(setting):
        got = {
            "single_f32": [t.cpu() for t in api.solve(qf, k=12)],
            "single_i32": [t.cpu() for t in api.solve(qi, k=7)],
            "batched_f32": [t.cpu() for t in api.solve_batched(bf, nsf, k=3)],
            "batched_i32": [t.cpu() for t in api.solve_batched(bi, nsi, k=64)],
        }
    for key in ref:
        for a, b in zip(got[key], ref[key]):
            assert torch.equal(a, b), (key, setting)
