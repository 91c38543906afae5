"""Second moments E_p[x_i x_j], marginals and E_p[f] of the Boltzmann
distribution p(x) = exp(-beta f(x) - logZ) from qubo_logz_moments, against
brute force over all states (oracle energies, float64) and the oracle's
gradient (G = -beta * moments).  Tolerance: max-norm relative 1e-4, as for
the gradient (same walk, same float32 block sums)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2310_19373_amd import api, inputs

pytestmark = pytest.mark.gpu


def _brute(Q, beta):
    n = Q.shape[0]
    masks = np.arange(1 << n, dtype=np.uint64)
    E = oracle.energies(Q, masks)
    a = -beta * E
    w = np.exp(a - a.max())
    p = w / w.sum()
    X = ((masks[:, None] >> np.arange(n, dtype=np.uint64)) & np.uint64(1)).astype(np.float64)
    M = np.triu((X * p[:, None]).T @ X)
    return M, float(p @ E)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


@pytest.mark.parametrize("beta", [0.0, 1.3, -2.0, 6.0])
@pytest.mark.parametrize("n", [1, 5, 12])
def test_moments_brute_force(gpu_lib, n, beta):
    Q = inputs.random_f32(n, 700 + n, scale=1 / math.sqrt(n))
    print(f"moments n={n} beta={beta}", flush=True)
    lz, M, mean = api.logz_moments(Q, beta)
    Mref, mref = _brute(Q, beta)
    M = M.cpu().numpy()
    assert _rel(M, Mref) <= 1e-4
    assert np.all(np.tril(M, -1) == 0)
    assert abs(float(mean) - mref) <= 1e-4 * max(1.0, abs(mref))
    if beta == 0.0:
        assert np.allclose(np.diag(M), 0.5, atol=1e-6) and np.allclose(M[np.triu_indices(n, 1)], 0.25, atol=1e-6)


def test_moments_match_oracle_gradient(gpu_lib):
    Q = inputs.random_f32(18, 710, scale=1 / math.sqrt(18))
    beta = 2.5
    lz, M, mean = api.logz_moments(Q, beta)
    ref, mref = oracle.logz(Q, beta, with_mean=True)
    assert abs(float(lz) - ref) <= 2e-6 + 4e-7 * beta * float(np.abs(Q.astype(np.float64)).sum())
    G = oracle.grad(Q, beta, ref)
    assert _rel(M.cpu().numpy(), G / -beta) <= 1e-4
    assert abs(float(mean) - mref) <= 1e-4 * max(1.0, abs(mref))
    marg = api.marginals(Q, beta).cpu().numpy()
    assert _rel(marg, np.diag(G) / -beta) <= 1e-4


def test_moments_batched_padding(gpu_lib):
    rng = np.random.default_rng(720)
    batch, nmax = 10, 16
    ns = rng.integers(1, nmax + 1, batch).astype(np.int32)
    betas = rng.choice([0.0, 0.5, -1.5, 3.0], batch).astype(np.float32)
    Q = np.zeros((batch, nmax, nmax), dtype=np.float32)
    for b, n in enumerate(ns):
        Q[b, :n, :n] = np.triu(rng.normal(0, 1 / math.sqrt(n), (n, n))).astype(np.float32)
    lz, M, mean = api.logz_moments(torch.from_numpy(Q), torch.from_numpy(betas), ns=torch.from_numpy(ns))
    M = M.cpu().numpy()
    for b, n in enumerate(ns):
        Mref, mref = _brute(np.ascontiguousarray(Q[b, :n, :n]), float(betas[b]))
        assert _rel(M[b, :n, :n], Mref) <= 1e-4, b
        assert np.all(M[b, n:, :] == 0) and np.all(M[b, :, n:] == 0), b
        assert abs(float(mean[b]) - mref) <= 1e-4 * max(1.0, abs(mref)), b


def test_moments_n32_diagonal_closed_form(gpu_lib):
    # n = 32: independent bits, E[x_i] = p_i, E[x_i x_j] = p_i p_j, E[f] = sum d_i p_i
    n, beta = 32, 1.1
    d = np.linspace(-1.5, 2.5, n).astype(np.float32)
    lz, M, mean = api.logz_moments(np.diag(d), beta)
    p = 1.0 / (1.0 + np.exp(beta * d.astype(np.float64)))
    ref = np.triu(np.outer(p, p), 1) + np.diag(p)
    assert _rel(M.cpu().numpy(), ref) <= 1e-4
    assert abs(float(mean) - float(d.astype(np.float64) @ p)) <= 1e-4 * max(1.0, abs(float(d @ p)))
