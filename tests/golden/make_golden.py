"""Write the stored expected values under tests/golden/ by calling only the
CPU oracle on the seeded workloads.

    python tests/golden/make_golden.py [name ...]

Names: single_n20_f32, single_n32_i32, single_n40_f32_planted, logz_sample,
batched_sample, batched_mid, single_mid_f32, logz_general.  Each JSON file records the workload, the oracle call, the
host thread count and the wall time.  Float energies are stored as Python
float reprs (exact round trip of the float64 value).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2310_19373_amd import inputs  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def _dump(name, payload):
    path = os.path.join(OUT, name + ".json")
    with open(path, "w") as f:
        json.dump(payload, f, indent=1)
        f.write("\n")
    print("wrote", path, flush=True)


def _energies(E):
    return [int(e) if isinstance(e, (np.integer, int)) else float(e) for e in E.tolist()]


def single_n20_f32():
    Q = inputs.single_n20_f32()
    t = time.time()
    E, M = oracle.topk(Q, 16)
    _dump("single_n20_f32", {
        "workload": "n=20 float32 N(0,1), seed 0 (natural-order brute force)",
        "call": "oracle.topk(Q, 16)", "threads": oracle.max_threads(), "seconds": time.time() - t,
        "energies": _energies(E), "masks": [int(m) for m in M]})


def single_n32_i32():
    Q = inputs.single_n32_i32()
    t = time.time()
    E, M = oracle.topk(Q, 32)
    _dump("single_n32_i32", {
        "workload": "n=32 int32 uniform [-100,100], seed 1 (natural-order brute force, int64)",
        "call": "oracle.topk(Q, 32)", "threads": oracle.max_threads(), "seconds": time.time() - t,
        "energies": _energies(E), "masks": [int(m) for m in M]})


def single_n40_f32_planted():
    Q, xstar = inputs.single_n40_f32_planted()
    e = oracle.energy(Q, xstar)
    # Sampled prefix ranges: the full top-k of 8 random ranges of 2^22 masks.
    rng = np.random.default_rng(40)
    ranges = []
    t = time.time()
    for p in rng.integers(0, 1 << 18, 8):
        lo = int(p) << 22
        E, M = oracle.topk(Q, 8, lo=lo, hi=lo + (1 << 22))
        ranges.append({"lo": lo, "hi": lo + (1 << 22), "energies": _energies(E), "masks": [int(m) for m in M]})
    t_random = time.time() - t
    # Ranges where the lowest states live: the aligned block of 2^22 masks that
    # holds the planted minimiser, and the blocks holding it with one of the
    # top 18 bits flipped (x* comes from the generator, not from any solve).
    near = []
    t = time.time()
    for h in [None] + list(range(22, 40)):
        x = int(xstar) if h is None else int(xstar) ^ (1 << h)
        lo = (x >> 22) << 22
        E, M = oracle.topk(Q, 16, lo=lo, hi=lo + (1 << 22))
        near.append({"lo": lo, "hi": lo + (1 << 22), "flipped_bit": h, "energies": _energies(E),
                     "masks": [int(m) for m in M]})
    _dump("single_n40_f32_planted", {
        "workload": "n=40 float32 N(0,1/n) + planted minimiser, seed 2",
        "xstar": int(xstar), "energy_xstar": float(e), "threads": oracle.max_threads(),
        "ranges_seconds": t_random, "ranges": ranges,
        "near_ranges_k": 16, "near_ranges_seconds": time.time() - t, "near_ranges": near})


def logz_sample():
    Q, beta = inputs.logz_256x24()
    picks = [0, 1, 2, 301, 767]
    rows = []
    t = time.time()
    for p in picks:
        lz, mean = oracle.logz(Q[p], float(beta[p]), with_mean=True)
        G = oracle.grad(Q[p], float(beta[p]), lz)
        rows.append({"pair": p, "beta": float(beta[p]), "logz": lz, "mean_energy": mean,
                     "grad_upper": [float(v) for v in G[np.triu_indices(24)]]})
    _dump("logz_sample", {
        "workload": "256 x n=24 float32 N(0,1/n), seed 4, beta in {0.5,1,4}; pair = 3*instance + beta index",
        "threads": oracle.max_threads(), "seconds": time.time() - t, "pairs": rows})


def batched_sample():
    Qp, ns = inputs.batched_4096()
    rng = np.random.default_rng(3)
    big = [int(b) for b in np.nonzero(ns >= 25)[0]]
    picks = sorted(int(b) for b in rng.choice(big, 6, replace=False))
    rows = []
    t = time.time()
    for b in picks:
        n = int(ns[b])
        E, M = oracle.topk(np.ascontiguousarray(Qp[b, :n, :n]), 2)
        rows.append({"instance": b, "n": n, "energies": _energies(E), "masks": [int(m) for m in M]})
    _dump("batched_sample", {
        "workload": "4096 instances, n_b uniform [12,28], N(0,1) float32, seed 3 (instances with n_b >= 25, sampled)",
        "threads": oracle.max_threads(), "seconds": time.time() - t, "instances": rows})


def batched_mid():
    # argmin and runner-up of 72 instances of the 4096-instance workload, six
    # for each n_b in 17..28 (the first six of that size in batch order)
    Qp, ns = inputs.batched_4096()
    picks = []
    for n in range(17, 29):
        picks += [int(b) for b in np.nonzero(ns == n)[0][:6]]
    rows = []
    t = time.time()
    for b in sorted(picks):
        n = int(ns[b])
        E, M = oracle.topk(np.ascontiguousarray(Qp[b, :n, :n]), 2)
        rows.append({"instance": b, "n": n, "energies": _energies(E), "masks": [int(m) for m in M]})
    _dump("batched_mid", {
        "workload": "4096 instances, n_b uniform [12,28], N(0,1) float32, seed 3 (six instances per n_b in 17..28)",
        "call": "oracle.topk(Q_b, 2)", "threads": oracle.max_threads(), "seconds": time.time() - t,
        "instances": rows})


SINGLE_MID = [(27, 2700), (28, 2800), (29, 2900), (30, 3000), (31, 3100)]


def single_mid_f32():
    # single float32 solves at the sizes where the single-solve bit split
    # changes (unit bits 9..11), N(0,1) entries
    rows = []
    t = time.time()
    for n, seed in SINGLE_MID:
        Q = inputs.random_f32(n, seed)
        E, M = oracle.topk(Q, 16)
        rows.append({"n": n, "seed": seed, "energies": _energies(E), "masks": [int(m) for m in M]})
        print("  n", n, time.time() - t, flush=True)
    _dump("single_mid_f32", {
        "workload": "float32 N(0,1), inputs.random_f32(n, seed), k=16 (natural-order brute force)",
        "call": "oracle.topk(Q, 16)", "threads": oracle.max_threads(), "seconds": time.time() - t,
        "instances": rows})


LOGZ_GENERAL = [(28, 2801, 0.5), (28, 2801, 4.0), (32, 3201, 0.5), (32, 3201, 4.0)]


def logz_general():
    # logZ, E_p[f] and the gradient of general Q (N(0, 1/n) float32 entries) at
    # the largest sizes the log-partition calls take
    rows = []
    t = time.time()
    for n, seed, beta in LOGZ_GENERAL:
        Q = inputs.random_f32(n, seed, scale=1 / np.sqrt(n))
        lz, mean = oracle.logz(Q, beta, with_mean=True)
        G = oracle.grad(Q, beta, lz)
        rows.append({"n": n, "seed": seed, "beta": beta, "logz": lz, "mean_energy": mean,
                     "grad_upper": [float(v) for v in G[np.triu_indices(n)]]})
        print("  n", n, "beta", beta, time.time() - t, flush=True)
    _dump("logz_general", {
        "workload": "float32 N(0,1/n), inputs.random_f32(n, seed, scale=1/sqrt(n)); logZ two-pass Neumaier, "
                    "gradient Neumaier sum of p(x) x_i x_j",
        "call": "oracle.logz(Q, beta, with_mean=True); oracle.grad(Q, beta, logz)",
        "threads": oracle.max_threads(), "seconds": time.time() - t, "pairs": rows})


ALL = {f.__name__: f for f in (single_n20_f32, single_n32_i32, single_n40_f32_planted, logz_sample,
                               batched_sample, batched_mid, single_mid_f32, logz_general)}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(ALL)):
        ALL[name]()
