"""Seeded synthetic QUBO instances.

This module only draws numbers: it evaluates no energy, walks no state space
and shares nothing with either the HIP path or the CPU oracle, both of which
consume the arrays it returns.  Every recipe uses numpy's PCG64 generator
(``numpy.random.default_rng(seed)``), draws the full n x n matrix, keeps the
upper triangle (the objective of Eq. 1 reads only entries with i <= j) and
casts to the stored dtype.  The paper states no instance distribution beyond
"random QUBO instances" (Sec. 3, timing experiment), so these recipes stand in
for its workloads.

Named workloads (n, dtype, seed):

* ``single_n20_f32``   n=20, N(0,1) float32, seed 0, k=8
* ``single_n32_i32``   n=32, uniform integers in [-100, 100], seed 1, k=16
* ``single_n40_f32_planted``  n=40, N(0, 1/n) float32 with a planted unique
  minimiser (margin >= 1), seed 2, k=16
* ``batched_4096``     4096 instances, n_b uniform in [12, 28], N(0,1) float32,
  seed 3, zero-padded to [4096, 28, 28]
* ``logz_256x24``      256 instances, n=24, N(0, 1/n) float32, seed 4, each
  paired with beta in {0.5, 1, 4} (768 pairs)
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "random_f32",
    "random_i32",
    "planted_f32",
    "single_n20_f32",
    "single_n32_i32",
    "single_n40_f32_planted",
    "batched_4096",
    "logz_256x24",
    "LOGZ_BETAS",
]

LOGZ_BETAS = (0.5, 1.0, 4.0)


def random_f32(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Upper-triangular float32 Q with i.i.d. N(0, scale^2) entries."""
    rng = np.random.default_rng(seed)
    q = rng.normal(0.0, scale, (n, n)) if scale != 1.0 else rng.standard_normal((n, n))
    return np.triu(q).astype(np.float32)


def random_i32(n: int, seed: int, lo: int = -100, hi: int = 100) -> np.ndarray:
    """Upper-triangular int32 Q with entries uniform in [lo, hi] (inclusive)."""
    rng = np.random.default_rng(seed)
    return np.triu(rng.integers(lo, hi + 1, (n, n), dtype=np.int32))


def _plant(q: np.ndarray, xstar: np.ndarray, slack: float = 1e-3) -> np.ndarray:
    """Shift the diagonal so that ``xstar`` is the unique minimiser by >= 1.

    For x = xstar with the bits of a nonempty set D flipped, the original
    objective can drop by at most sum_{i in D} R_i, where R_i = |Q_ii| plus the
    absolute off-diagonal entries of row and column i.  Adding
    lambda_i * (1 - 2 xstar_i) to Q_ii, with lambda_i = R_i + 1 + slack, raises
    the objective of every such x by sum_{i in D} lambda_i, so each competitor
    lies at least |D| + slack*|D| above xstar.  R is taken in float64 from the
    stored float32 values; the slack absorbs the final rounding of the shifted
    diagonal to float32.
    """
    n = q.shape[0]
    q64 = q.astype(np.float64)
    off = np.triu(q64, 1)
    sym = off + off.T
    r = np.abs(np.diag(q64)) + np.abs(sym).sum(axis=1)
    lam = r + 1.0 + slack
    out = q64.copy()
    out[np.arange(n), np.arange(n)] += lam * (1.0 - 2.0 * xstar.astype(np.float64))
    return out.astype(np.float32)


def planted_f32(n: int, seed: int):
    """N(0, 1/n) float32 Q with a planted minimiser; returns (Q, xstar_mask)."""
    rng = np.random.default_rng(seed)
    q = np.triu(rng.normal(0.0, 1.0 / np.sqrt(n), (n, n))).astype(np.float32)
    xstar = rng.integers(0, 2, n)
    qp = _plant(q, xstar)
    mask = 0
    for i in range(n):
        if xstar[i]:
            mask |= 1 << i
    return qp, mask


def single_n20_f32():
    return random_f32(20, 0)


def single_n32_i32():
    return random_i32(32, 1)


def single_n40_f32_planted():
    return planted_f32(40, 2)


def batched_4096(batch: int = 4096, nlo: int = 12, nhi: int = 28, seed: int = 3):
    """Returns (Qpad [batch, nhi, nhi] float32, ns [batch] int32)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nlo, nhi + 1, batch)
    qpad = np.zeros((batch, nhi, nhi), dtype=np.float32)
    for b in range(batch):
        nb = int(ns[b])
        qpad[b, :nb, :nb] = np.triu(rng.standard_normal((nb, nb))).astype(np.float32)
    return qpad, ns.astype(np.int32)


def logz_256x24(count: int = 256, n: int = 24, seed: int = 4):
    """Returns (Q [count*3, n, n] float32, beta [count*3] float32).

    Instance c is repeated for the three betas, so pair index = 3*c + i.
    """
    rng = np.random.default_rng(seed)
    qs = np.stack([np.triu(rng.normal(0.0, 1.0 / np.sqrt(n), (n, n))).astype(np.float32)
                   for _ in range(count)])
    q = np.repeat(qs, len(LOGZ_BETAS), axis=0)
    beta = np.tile(np.asarray(LOGZ_BETAS, dtype=np.float32), count)
    return q, beta
