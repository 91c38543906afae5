"""Batched solves on the GPU against the CPU oracle and against single solves;
HIP-graph replays against the eager result."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2310_19373_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mixed_batch(batch, nlo, nhi, seed, dtype):
    rng = np.random.default_rng(seed)
    ns = rng.integers(nlo, nhi + 1, batch).astype(np.int32)
    Q = np.zeros((batch, nhi, nhi), dtype=np.float32 if dtype == "f32" else np.int32)
    for b in range(batch):
        n = int(ns[b])
        if dtype == "f32":
            Q[b, :n, :n] = np.triu(rng.standard_normal((n, n))).astype(np.float32)
        else:
            Q[b, :n, :n] = np.triu(rng.integers(-100, 101, (n, n)))
    return Q, ns


def _oracle_all(Q, ns, k):
    outE, outM = [], []
    for b in range(len(ns)):
        n = int(ns[b])
        E, M = oracle.topk(np.ascontiguousarray(Q[b, :n, :n]), k)
        outE.append(E)
        outM.append(M)
    return np.stack(outE), np.stack(outM)


@pytest.mark.parametrize("dtype", ["f32", "i32"])
@pytest.mark.parametrize("k", [1, 4])
def test_batched_uneven_sizes_against_oracle(gpu_lib, dtype, k):
    from paper_2310_19373_amd import api

    Q, ns = _mixed_batch(96, 1, 21, 41 + k, dtype)
    print(f"batched dtype={dtype} k={k} batch=96", flush=True)
    e, m = api.solve_batched(Q, ns, k)
    E, M = _oracle_all(Q, ns, k)
    assert np.array_equal(m.cpu().numpy().astype(np.uint64), M)
    assert np.array_equal(e.cpu().numpy(), E)


def test_batched_equals_single_solves(gpu_lib):
    from paper_2310_19373_amd import api

    Q, ns = _mixed_batch(12, 18, 24, 77, "f32")
    e, m = api.solve_batched(Q, ns, 3)
    for b in range(12):
        n = int(ns[b])
        es, ms = api.solve(Q[b, :n, :n], 3)
        assert torch.equal(es, e[b]) and torch.equal(ms, m[b]), b


def test_batched_bad_size_status(gpu_lib):
    from paper_2310_19373_amd import api

    Q, ns = _mixed_batch(5, 4, 10, 5, "f32")
    ns[2] = 0
    with pytest.raises(api.QuboError) as ei:
        api.solve_batched(Q, ns, 1)
    assert ei.value.code == -1


def test_batched_config4_against_oracle(gpu_lib):
    # 4096 instances, n uniform in [12, 28]: all instances with n <= 16 are
    # compared live, the sampled n >= 25 instances against stored oracle values.
    from paper_2310_19373_amd import api

    Q, ns = inputs.batched_4096()
    print("batched config: 4096 instances n in [12, 28]", flush=True)
    e, m = api.solve_batched(Q, ns, 1)
    e, m = e.cpu().numpy(), m.cpu().numpy().astype(np.uint64)
    small = np.nonzero(ns <= 16)[0]
    for b in small:
        n = int(ns[b])
        E, M = oracle.topk(np.ascontiguousarray(Q[b, :n, :n]), 1)
        assert m[b, 0] == M[0] and e[b, 0] == E[0], b
    g = json.load(open(os.path.join(GOLDEN, "batched_sample.json")))
    for row in g["instances"]:
        b = row["instance"]
        assert int(m[b, 0]) == row["masks"][0] and e[b, 0] == row["energies"][0], b
    # every returned energy is the oracle energy of the returned mask
    pick = np.random.default_rng(0).choice(len(ns), 64, replace=False)
    for b in pick:
        n = int(ns[b])
        assert e[b, 0] == oracle.energy(np.ascontiguousarray(Q[b, :n, :n]), int(m[b, 0]))


def test_graph_replays_match_eager(gpu_lib):
    from paper_2310_19373_amd import api

    Q, ns = _mixed_batch(64, 8, 22, 99, "f32")
    eager = api.BatchedSolver(64, 22, 2)
    eager.load(Q, ns)
    eager.run()
    e0, m0 = [t.clone() for t in eager.results()]
    g = api.BatchedSolver(64, 22, 2, graph=True)
    g.load(Q, ns)
    for rep in range(4):
        g.energies.fill_(0)
        g.masks.fill_(0)
        g.run()
        torch.cuda.synchronize()
        e, m = g.results()
        assert torch.equal(e, e0) and torch.equal(m, m0), rep
        # the program's own eager work between replays
        eager.run()
        torch.cuda.synchronize()
    # new inputs through the same captured graph
    Q2, ns2 = _mixed_batch(64, 8, 22, 100, "f32")
    g.load(Q2, ns2)
    g.run()
    torch.cuda.synchronize()
    e, m = g.results()
    E, M = _oracle_all(Q2, ns2, 2)
    assert np.array_equal(m.cpu().numpy().astype(np.uint64), M) and np.array_equal(e.cpu().numpy(), E)


def test_batched_config4_mid_sizes_against_golden(gpu_lib):
    # the same 4096-instance batch with k=2: six instances of every n_b in
    # 17..28 against their stored oracle top-2 (argmin and runner-up)
    from paper_2310_19373_amd import api

    Q, ns = inputs.batched_4096()
    print("batched config: 4096 instances, k=2", flush=True)
    e, m = api.solve_batched(Q, ns, 2)
    e, m = e.cpu().numpy(), m.cpu().numpy().astype(np.uint64)
    g = json.load(open(os.path.join(GOLDEN, "batched_mid.json")))
    assert len(g["instances"]) >= 64
    assert sorted({row["n"] for row in g["instances"]}) == list(range(17, 29))
    for row in g["instances"]:
        b = row["instance"]
        assert int(ns[b]) == row["n"], b
        assert [int(x) for x in m[b]] == row["masks"], b
        assert e[b].tolist() == row["energies"], b
