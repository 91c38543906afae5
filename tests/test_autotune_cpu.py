"""Host logic of the autotuner: the search, the signature and the cache."""
import json

import numpy as np
import pytest

from paper_2310_19373_amd import _lib, autotune


def test_coordinate_descent_finds_separable_minimum():
    space = {"a": (1, 2, 3, 4), "b": (10, 20, 30)}
    calls = []

    def cost(s):
        calls.append(dict(s))
        return (s["a"] - 3) ** 2 + (s["b"] - 20) ** 2 / 100.0

    best, c, trials = autotune.coordinate_descent(space, {"a": 1, "b": 30}, cost)
    assert best == {"a": 3, "b": 20}
    assert c == 0.0
    keys = [tuple(sorted(s.items())) for s in calls]
    assert len(keys) == len(set(keys)), "a setting was evaluated twice"
    assert trials[0] == ({"a": 1, "b": 30}, 1**2 * 4 + 1.0)


def test_coordinate_descent_skips_rejected_settings():
    space = {"a": (1, 2, 3)}

    def cost(s):
        return None if s["a"] == 3 else -s["a"]

    best, c, trials = autotune.coordinate_descent(space, {"a": 1}, cost)
    assert best == {"a": 2} and c == -2
    assert ({"a": 3}, None) in trials


def test_coordinate_descent_rejected_start_raises():
    with pytest.raises(RuntimeError):
        autotune.coordinate_descent({"a": (1, 2)}, {"a": 1}, lambda s: None)


def test_signature_and_cache_roundtrip(tmp_path):
    ns = np.array([12, 12, 20, 28], dtype=np.int32)
    sig = autotune.batched_signature(ns, 1, "f32", "dev")
    assert sig["batch"] == 4 and sig["nmax"] == 28
    assert sig["states"] == 2 * 2.0**12 + 2.0**20 + 2.0**28
    assert sig["n_hist"] == {"12": 2, "20": 1, "28": 1}
    path = str(tmp_path / "tune.json")
    assert autotune.load_cached(path, sig) is None
    autotune.save_cached(path, sig, {"batched_outer": 7}, 1.5)
    assert autotune.load_cached(path, sig) == {"batched_outer": 7}
    other = dict(sig, k=2)
    assert autotune.load_cached(path, other) is None
    with open(path) as f:
        assert len(json.load(f)) == 1


def test_knobs_apply_and_restore():
    names = ["batched_outer", "waves_per_cu", "chunk_batched"]
    before = autotune.current(names)
    with autotune.keep_tuning(names):
        autotune.apply({"batched_outer": 7, "waves_per_cu": 8, "chunk_batched": 2})
        assert autotune.current(names) == {"batched_outer": 7, "waves_per_cu": 8, "chunk_batched": 2}
    assert autotune.current(names) == before


def test_every_search_value_is_accepted_by_the_library():
    for space in (autotune.BATCHED_SPACE, autotune.SINGLE_SPACE):
        names = list(space)
        with autotune.keep_tuning(names):
            for nm, values in space.items():
                for v in values:
                    autotune.apply({nm: v})
                    assert _lib.get_tuning(autotune.KNOBS[nm]) == v, (nm, v)
