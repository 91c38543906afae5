"""The autotuner on the GPU: it measures, keeps outputs identical, applies."""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_19373_amd import api, autotune

pytestmark = pytest.mark.gpu

SPACE = {"batched_outer": (6, 8), "waves_per_cu": (8, 12), "chunk_batched": (2, 8)}


def _batch(seed=11, batch=96, lo=12, hi=20):
    rng = np.random.default_rng(seed)
    ns = rng.integers(lo, hi + 1, batch).astype(np.int32)
    q = np.zeros((batch, hi, hi), dtype=np.float32)
    for b, n in enumerate(ns):
        q[b, :n, :n] = np.triu(rng.standard_normal((n, n))).astype(np.float32)
    return q, ns


def test_tune_batched_applies_best_and_keeps_results(tmp_path):
    q, ns = _batch()
    names = list(SPACE)
    with autotune.keep_tuning(names):
        res = autotune.tune_batched(q, ns, k=1, space=SPACE, reps=2, cache=str(tmp_path / "t.json"))
        print("tuned", res.best, res.ms, "start", res.start, res.start_ms, flush=True)
        assert set(res.best) == set(SPACE)
        for nm, v in res.best.items():
            assert v in SPACE[nm] or v == res.start[nm]
        assert res.ms <= res.start_ms
        assert autotune.current(names) == res.best
        assert all(c is not None for _, c, _ in res.trials), "a setting changed the results"
        en, mk = api.solve_batched(q, ns, k=1)
        en, mk = en.cpu().numpy(), mk.cpu().numpy()
        for b in range(0, len(ns), 7):
            n = int(ns[b])
            oe, om = oracle.topk(q[b, :n, :n], 1)
            assert mk[b, 0] == om[0]
            assert abs(en[b, 0] - oe[0]) <= 1e-9 * max(abs(oe[0]), 1e-12)
        assert autotune.load_cached(str(tmp_path / "t.json"), res.signature) == res.best


def test_tune_without_apply_restores_knobs():
    q, ns = _batch(seed=12, batch=32)
    names = list(SPACE)
    before = autotune.current(names)
    autotune.tune_batched(q, ns, k=1, space={"batched_outer": (6,)}, reps=1, apply_best=False)
    assert autotune.current(names) == before


def test_tune_single_small():
    rng = np.random.default_rng(5)
    q = np.triu(rng.standard_normal((24, 24))).astype(np.float32)
    space = {"single_outer": (8, 10), "chunk_single": (1, 4)}
    with autotune.keep_tuning(space):
        res = autotune.tune_single(q, k=4, space=space, reps=1)
        assert res.ms <= res.start_ms
        en, mk = api.solve(q, k=4)
        oe, om = oracle.topk(q, 4)
        assert [int(m) for m in mk.cpu().numpy()] == [int(m) for m in om]
