"""Log-partition function and its gradient on the GPU against the CPU oracle.

Tolerances (derived from the float32 walk arithmetic; u = 2^-24):
  logZ: each state's exponent is formed from float32 table values and a float32
  fma, so its error is at most about 3u*|beta|*sum|Q| (table rounding, the
  sum and the per-step constant); the weights are summed in float32 over at
  most 16 steps per entry (matrix-core accumulation), folded in chains of 8
  products summed pairwise, then in float64: at most about 26u ~ 1.6e-6
  relative, all terms positive, plus exp2's error.  The test allows
  |dlogZ| <= 2e-6 + 4e-7 * |beta| * sum|Q|.
  gradient: max-norm relative error <= 1e-4 against the float64 oracle.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2310_19373_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def logz_tol(Q, beta):
    return 2e-6 + 4e-7 * abs(beta) * float(np.abs(np.triu(Q.astype(np.float64))).sum())


def _gpu_logz_grad(Q, beta):
    from paper_2310_19373_amd import api

    print(f"logz n={Q.shape[0]} beta={beta}", flush=True)
    Qt = torch.from_numpy(Q).cuda().requires_grad_(True)
    bt = torch.tensor(float(beta), dtype=torch.float32, device="cuda", requires_grad=True)
    lz = api.logz(Qt, bt)
    lz.backward()
    return float(lz.detach()), Qt.grad.cpu().numpy().astype(np.float64), float(bt.grad)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


@pytest.mark.parametrize("n", [1, 3, 5, 6, 10, 11, 12, 15, 18])
@pytest.mark.parametrize("beta", [0.5, 1.0, 4.0, -0.7])
def test_logz_and_grad_against_oracle(gpu_lib, n, beta):
    Q = inputs.random_f32(n, 800 + n, scale=1 / math.sqrt(n))
    lz, G, gb = _gpu_logz_grad(Q, beta)
    ref, mean = oracle.logz(Q, beta, with_mean=True)
    assert abs(lz - ref) <= logz_tol(Q, beta), (lz, ref)
    Gref = oracle.grad(Q, beta, ref)
    assert _rel(G, Gref) <= 1e-4
    assert np.all(np.tril(G, -1) == 0)
    assert abs(gb + mean) <= 1e-4 * max(1.0, abs(mean))


def test_logz_beta_zero_and_zero_matrix(gpu_lib):
    Q = inputs.random_f32(13, 5)
    lz, G, gb = _gpu_logz_grad(Q, 0.0)
    assert abs(lz - 13 * math.log(2)) < 1e-9
    assert np.all(G == 0)
    Z = np.zeros((9, 9), dtype=np.float32)
    lz, G, gb = _gpu_logz_grad(Z, 1.5)
    assert abs(lz - 9 * math.log(2)) < 1e-9
    iu = np.triu_indices(9, 1)
    np.testing.assert_allclose(np.diag(G), -1.5 / 2, rtol=1e-6)
    np.testing.assert_allclose(G[iu], -1.5 / 4, rtol=1e-6)


def test_logz_diagonal_closed_form(gpu_lib):
    d = np.random.default_rng(3).normal(0, 1, 14).astype(np.float32)
    Q = np.diag(d).astype(np.float32)
    beta = 1.7
    lz, G, gb = _gpu_logz_grad(Q, beta)
    ref = sum(math.log1p(math.exp(-beta * float(v))) for v in d)
    assert abs(lz - ref) <= logz_tol(Q, beta)
    sig = 1.0 / (1.0 + np.exp(beta * d.astype(np.float64)))
    np.testing.assert_allclose(np.diag(G), -beta * sig, rtol=1e-4, atol=1e-7)
    iu = np.triu_indices(14, 1)
    np.testing.assert_allclose(G[iu], (-beta * np.outer(sig, sig))[iu], rtol=1e-4, atol=1e-7)


def test_grad_against_central_differences(gpu_lib):
    # central differences of the float64 oracle logZ (h = 1e-3) vs the GPU adjoint
    n = 9
    Q = inputs.random_f32(n, 61, scale=1 / math.sqrt(n))
    beta = 1.0
    _, G, _ = _gpu_logz_grad(Q, beta)
    Qd = Q.astype(np.float64)
    X = ((np.arange(1 << n)[:, None] >> np.arange(n)) & 1).astype(np.float64)

    def lz(Qm):
        a = -beta * np.einsum("bi,ij,bj->b", X, np.triu(Qm), X)
        m = a.max()
        return m + math.log(np.exp(a - m).sum())

    h = 1e-3
    fd = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            P = Qd.copy()
            P[i, j] += h
            M = Qd.copy()
            M[i, j] -= h
            fd[i, j] = (lz(P) - lz(M)) / (2 * h)
    assert _rel(G, fd) <= 1e-4


def test_batched_padded_logz(gpu_lib):
    from paper_2310_19373_amd import api

    rng = np.random.default_rng(12)
    batch, nmax = 24, 16
    ns = rng.integers(1, nmax + 1, batch).astype(np.int32)
    Q = np.zeros((batch, nmax, nmax), dtype=np.float32)
    betas = rng.choice([0.5, 1.0, 4.0, -2.0], batch).astype(np.float32)
    for b in range(batch):
        n = int(ns[b])
        Q[b, :n, :n] = np.triu(rng.normal(0, 1 / math.sqrt(n), (n, n))).astype(np.float32)
    Qt = torch.from_numpy(Q).cuda().requires_grad_(True)
    bt = torch.from_numpy(betas).cuda().requires_grad_(True)
    lz = api.logz(Qt, bt, ns=torch.from_numpy(ns))
    (lz * torch.arange(1, batch + 1, device="cuda", dtype=torch.float64)).sum().backward()
    G = Qt.grad.cpu().numpy()
    for b in range(batch):
        n = int(ns[b])
        Qb = np.ascontiguousarray(Q[b, :n, :n])
        ref = oracle.logz(Qb, float(betas[b]))
        assert abs(float(lz[b].detach()) - ref) <= logz_tol(Qb, float(betas[b])), b
        Gref = (b + 1) * oracle.grad(Qb, float(betas[b]), ref)
        assert _rel(G[b, :n, :n].astype(np.float64), Gref) <= 1e-4, b
        assert np.all(G[b, n:, :] == 0) and np.all(G[b, :, n:] == 0)


def test_logz_config_sample(gpu_lib):
    # 256 x n=24 instances x beta in {0.5, 1, 4}: sampled pairs against stored
    # oracle values; all pairs: convexity in beta and moment bounds.
    from paper_2310_19373_amd import api

    Q, beta = inputs.logz_256x24()
    Qt = torch.from_numpy(Q).cuda().requires_grad_(True)
    bt = torch.from_numpy(beta).cuda()
    print("logz config: 768 pairs n=24", flush=True)
    lz = api.logz(Qt, bt)
    lz.sum().backward()
    lzc = lz.detach().cpu().numpy()
    G = Qt.grad.cpu().numpy().astype(np.float64)
    g = json.load(open(os.path.join(GOLDEN, "logz_sample.json")))
    iu = np.triu_indices(24)
    for row in g["pairs"]:
        p = row["pair"]
        assert abs(lzc[p] - row["logz"]) <= logz_tol(Q[p], row["beta"]), p
        Gref = np.zeros((24, 24))
        Gref[iu] = row["grad_upper"]
        assert _rel(G[p], Gref) <= 1e-4, p
    l3 = lzc.reshape(256, 3)
    # convexity: logZ(1) <= interpolation of logZ(0.5) and logZ(4)
    w = (4.0 - 1.0) / (4.0 - 0.5)
    assert np.all(l3[:, 1] <= w * l3[:, 0] + (1 - w) * l3[:, 2] + 1e-9)
    M = G / -beta[:, None, None]
    d = np.diagonal(M, axis1=1, axis2=2)
    off = M[:, iu[0], iu[1]]
    assert np.all(off >= -1e-6)
    assert np.all(off <= np.minimum(d[:, iu[0]], d[:, iu[1]]) + 1e-6)


def test_nonfinite_beta_flags_only_that_instance(gpu_lib):
    # beta = NaN or inf: that instance's status is QUBO_ERR_NONFINITE and its
    # logZ NaN; the other instances of the batch are unaffected
    from paper_2310_19373_amd import _lib

    batch, n = 4, 10
    Q = np.stack([inputs.random_f32(n, 1800 + b, scale=0.3) for b in range(batch)])
    betas = np.array([1.0, np.nan, np.inf, -0.5], dtype=np.float32)
    Qd = torch.from_numpy(Q).cuda()
    bd = torch.from_numpy(betas).cuda()
    nsd = torch.full((batch,), n, dtype=torch.int32, device="cuda")
    L = _lib.lib()
    wsb = L.qubo_logz_workspace_size(batch, n)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    lz = torch.empty(batch, dtype=torch.float64, device="cuda")
    st = torch.empty(batch, dtype=torch.int32, device="cuda")
    _lib.check(L.qubo_logz_fwd(batch, Qd.data_ptr(), n, nsd.data_ptr(), bd.data_ptr(), lz.data_ptr(), st.data_ptr(),
                               ws.data_ptr(), wsb, None))
    torch.cuda.synchronize()
    assert st.cpu().tolist() == [0, _lib.QUBO_ERR_NONFINITE, _lib.QUBO_ERR_NONFINITE, 0]
    lz = lz.cpu().numpy()
    assert np.isnan(lz[1]) and np.isnan(lz[2])
    for b in (0, 3):
        assert abs(lz[b] - oracle.logz(Q[b], float(betas[b]))) <= logz_tol(Q[b], float(betas[b]))


def test_logz_rejects_a_nonzero_lower_triangle(gpu_lib):
    from paper_2310_19373_amd import api

    Q = inputs.random_f32(10, 870, scale=0.3)
    full = Q + np.tril(np.full((10, 10), 0.25, dtype=np.float32), -1)
    with pytest.raises(ValueError):
        api.logz(torch.from_numpy(full).cuda(), 1.0)
    # opted out: the lower triangle is ignored, as by the C ABI
    lz = float(api.logz(torch.from_numpy(full).cuda(), 1.0, check_lower=False))
    assert lz == float(api.logz(torch.from_numpy(Q).cuda(), 1.0))
    assert abs(lz - oracle.logz(Q, 1.0)) <= logz_tol(Q, 1.0)



def test_logz_general_q_at_28_and_32_against_golden(gpu_lib):
    # general Q (N(0, 1/n)) at the largest log-partition sizes, where each
    # lane's float32 sums inside a work unit are longest: stored float64 oracle
    # logZ, E_p[f] and gradient
    g = json.load(open(os.path.join(GOLDEN, "logz_general.json")))
    assert sorted({row["n"] for row in g["pairs"]}) == [28, 32]
    for row in g["pairs"]:
        n, beta = row["n"], row["beta"]
        Q = inputs.random_f32(n, row["seed"], scale=1 / math.sqrt(n))
        lz, G, gb = _gpu_logz_grad(Q, beta)
        Gref = np.zeros((n, n))
        Gref[np.triu_indices(n)] = row["grad_upper"]
        err = _rel(G, Gref)
        print(f"  n={n} beta={beta}: |dlogZ| {abs(lz - row['logz']):.3e}, grad max-norm rel {err:.3e}, "
              f"dlogZ/dbeta rel {abs(gb + row['mean_energy']) / max(1.0, abs(row['mean_energy'])):.3e}", flush=True)
        assert abs(lz - row["logz"]) <= logz_tol(Q, beta), (n, beta)
        assert err <= 1e-4, (n, beta, err)
        assert abs(gb + row["mean_energy"]) <= 1e-4 * max(1.0, abs(row["mean_energy"])), (n, beta)
