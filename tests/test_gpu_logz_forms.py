"""The forms of the log-partition walks (factored: one FMA per state; direct:
one exp2 per state) against the CPU oracle, and against each other.

The factored form is taken per work unit when |beta| log2(e) times the
lane's range of inner-table values is at most 84; large |beta| or large
entries push units to the direct form, so the large-beta cases below run a
mix of both.  Within the factored form the gradient walk evaluates its block
sums nested over the inner bits where every step's factor row has
b(t, 0) >= 2^-40 (knob value 1, the default), else with per-state products
(knob value 2 forces those everywhere).  logZ tolerance as in test_gpu_logz.py.  Gradient: a state's
exponent carries up to about 3u |beta| sum|Q| of float32 rounding (u = 2^-24),
which is also the relative error of its weight; at the large |beta| used here
that term is added to the 1e-4 max-norm bound (at beta <= 4 and N(0, 1/n)
entries it is below 4e-5).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2310_19373_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def logz_tol(Q, beta):
    return 2e-6 + 4e-7 * abs(beta) * float(np.abs(np.triu(Q.astype(np.float64))).sum())


def grad_tol(Q, beta):
    return 1e-4 + 2e-7 * abs(beta) * float(np.abs(np.triu(Q.astype(np.float64))).sum())


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


FORMS = {"nested": 1, "products": 2, "direct": -1}


def _run(Q, beta, form: str):
    from paper_2310_19373_amd import api

    old = _lib.get_tuning(_lib.TUNE_LOGZ_FACTORED)
    _lib.set_tuning(_lib.TUNE_LOGZ_FACTORED, FORMS[form])
    try:
        print(f"logz form={form} n={Q.shape[-1]} beta={beta}", flush=True)
        Qt = torch.from_numpy(Q).cuda().requires_grad_(True)
        bt = torch.tensor(float(beta), dtype=torch.float32, device="cuda", requires_grad=True)
        lz = api.logz(Qt, bt)
        lz.backward()
        return float(lz.detach()), Qt.grad.cpu().numpy().astype(np.float64), float(bt.grad)
    finally:
        _lib.set_tuning(_lib.TUNE_LOGZ_FACTORED, old)


CASES = [
    (12, 1.0, "scaled"), (18, 4.0, "scaled"), (20, 0.5, "scaled"), (22, 1.0, "scaled"),
    (16, 30.0, "unit"), (20, -25.0, "unit"), (22, 8.0, "unit"), (14, 3.0, "unit"),
]


@pytest.mark.parametrize("n,beta,kind", CASES)
@pytest.mark.parametrize("form", list(FORMS))
def test_form_against_oracle(gpu_lib, n, beta, kind, form):
    scale = 1 / math.sqrt(n) if kind == "scaled" else 1.0
    Q = inputs.random_f32(n, 900 + n, scale=scale)
    lz, G, gb = _run(Q, beta, form)
    ref, mean = oracle.logz(Q, beta, with_mean=True)
    assert abs(lz - ref) <= logz_tol(Q, beta), (lz, ref)
    Gref = oracle.grad(Q, beta, ref)
    assert _rel(G, Gref) <= grad_tol(Q, beta)
    assert abs(gb + mean) <= grad_tol(Q, beta) * max(1.0, abs(mean))


def test_forms_agree_on_mixed_batch(gpu_lib):
    from paper_2310_19373_amd import api

    rng = np.random.default_rng(31)
    batch, nmax = 40, 20
    ns = rng.integers(8, nmax + 1, batch).astype(np.int32)
    Q = np.zeros((batch, nmax, nmax), dtype=np.float32)
    betas = rng.choice([0.3, 2.0, 12.0, -20.0, 60.0], batch).astype(np.float32)
    for b in range(batch):
        n = int(ns[b])
        Q[b, :n, :n] = np.triu(rng.standard_normal((n, n))).astype(np.float32)
    out = {}
    for form, value in FORMS.items():
        old = _lib.get_tuning(_lib.TUNE_LOGZ_FACTORED)
        _lib.set_tuning(_lib.TUNE_LOGZ_FACTORED, value)
        try:
            Qt = torch.from_numpy(Q).cuda().requires_grad_(True)
            lz = api.logz(Qt, torch.from_numpy(betas).cuda(), ns=torch.from_numpy(ns))
            lz.sum().backward()
            out[form] = (lz.detach().cpu().numpy(), Qt.grad.cpu().numpy().astype(np.float64))
        finally:
            _lib.set_tuning(_lib.TUNE_LOGZ_FACTORED, old)
    for b in range(batch):
        n = int(ns[b])
        Qb = np.ascontiguousarray(Q[b, :n, :n])
        tol = logz_tol(Qb, float(betas[b]))
        for form in FORMS:
            assert abs(out[form][0][b] - out["direct"][0][b]) <= 2 * tol, (b, form)
        if b % 5 == 0:
            ref = oracle.logz(Qb, float(betas[b]))
            Gref = oracle.grad(Qb, float(betas[b]), ref)
            for form in FORMS:
                assert abs(out[form][0][b] - ref) <= tol, (b, form)
                assert _rel(out[form][1][b, :n, :n], Gref) <= grad_tol(Qb, float(betas[b])), (b, form)


def test_nested_form_is_taken(gpu_lib):
    """At beta = 1 and N(0, 1/n) entries every unit passes the nested form's
    bound, so the default gradient differs in rounding from the per-state
    products and both meet the oracle's bound."""
    n, beta = 22, 1.0
    Q = inputs.random_f32(n, 4242, scale=1 / math.sqrt(n))
    _, Gn, _ = _run(Q, beta, "nested")
    _, Gp, _ = _run(Q, beta, "products")
    assert not np.array_equal(Gn, Gp)
    ref = oracle.logz(Q, beta)
    Gref = oracle.grad(Q, beta, ref)
    assert _rel(Gn, Gref) <= grad_tol(Q, beta)
    assert _rel(Gp, Gref) <= grad_tol(Q, beta)
