"""The half-width screen's error bound, checked numerically on the CPU.

The float32 walk may screen a block of 64 inner states in float16: each
state's value C'(j) + Tb(b) + Ta(a) (j = b | a << 4, T' = Tb + Ta linear in the
inner bits) is formed from float16 roundings of the values scaled by
hs = 2^s, where R_I hs lies in [2^12, 2^13) and R_I is the sum of |Q| over the
six inner rows.  The margin the screen adds to its threshold must cover the
distance between that float16 value and hs times the float32 screen's value
fl32(fl32(T') + fl32(C')): the kernels' bound is 5.01 * 2^-11 * R_I * hs
(five float16 roundings of partial sums of the inner rows, plus the float32
ones), against a margin of 2^-8 * R_I * hs.

Here C', Tb and Ta come from random instances (float64 sums of the stored
float32 Q under random prefix and outer assignments), the float16 chain is
evaluated with numpy float16 arithmetic in the kernels' order (round C' to
float32, scale exactly, round to float16; Tb and Ta from float64 through
float32 to float16; two float16 additions), and the largest error over all
64 states must stay within the bound, at magnitudes from 1e-30 to 1e30 and
with inner rows that are negligible, typical or dominant."""
import numpy as np
import pytest

from paper_2310_19373_amd import inputs


def _screen_errors(Q, rng, draws=24):
    n = Q.shape[0]
    Qd = np.triu(Q).astype(np.float64)
    S = Qd + np.triu(Qd, 1).T                      # symmetric, diagonal d
    d = np.diag(Qd).copy()
    np.fill_diagonal(S, 0.0)
    # R_I: |Q| over the inner rows, both triangles (row u < 6, every column)
    R = float(sum(abs(Qd[min(u, v), max(u, v)]) for u in range(6) for v in range(n)))
    if R == 0.0:
        return 0.0, 1.0
    e = int(np.frexp(R)[1])
    hexp = 13 - e
    hs = 2.0 ** hexp
    worst = 0.0
    j = np.arange(64)
    bits = (j[:, None] >> np.arange(6)) & 1        # [64, 6]
    EI = np.zeros(64)
    for u in range(6):
        EI += bits[:, u] * d[u]
        for w in range(u + 1, 6):
            EI += bits[:, u] * bits[:, w] * Qd[u, w]
    for _ in range(draws):
        x = rng.integers(0, 2, n)
        x[:6] = 0
        # split the outer bits in half: one half are "prefix" bits (fixed per
        # lane), the other "outer" bits (the step's Gray value)
        pre = np.zeros(n, bool)
        pre[6 + (n - 6) // 2:] = True
        cI = np.array([float(np.sum(S[u, pre] * x[pre])) for u in range(6)])
        H = np.array([float(np.sum(S[u, ~pre] * x[~pre])) for u in range(6)])
        C = EI + bits @ cI                           # C'(j), float64
        T = bits @ H                                 # T'(j), float64
        s32 = (np.float32(T) + np.float32(C)).astype(np.float64)   # the float32 screen
        # the half screen, in the kernels' order
        C16 = np.ldexp(np.float32(C), hexp).astype(np.float16)
        b, a = j & 15, j >> 4
        Tb = np.array([float(sum(H[u] for u in range(4) if (bb >> u) & 1)) for bb in range(16)])
        Ta = np.array([0.0, H[4], H[5], H[4] + H[5]])
        Tb16 = np.float32(Tb * hs).astype(np.float16)
        Ta16 = np.float32(Ta * hs).astype(np.float16)
        s16 = ((C16 + Tb16[b]) + Ta16[a]).astype(np.float64)
        assert np.all(np.isfinite(s16))
        worst = max(worst, float(np.max(np.abs(s16 - hs * s32))) / (R * hs))
    return worst, R * hs


@pytest.mark.parametrize("scale", [1e-30, 1e-6, 1.0, 1e6, 1e30])
@pytest.mark.parametrize("inner", [1e-4, 1.0, 1e4])
def test_float16_screen_error_within_bound(scale, inner):
    rng = np.random.default_rng(int(abs(np.log10(scale))) * 7 + int(np.log10(inner)) + 50)
    for n in (14, 20):
        Q = inputs.random_f32(n, 5000 + n, scale=1.0).astype(np.float64)
        Q[:6, :] *= inner
        Q = (Q * scale).astype(np.float32)
        worst, Rs = _screen_errors(Q, rng)
        assert 2**12 <= Rs < 2**13
        assert worst <= 5.01 * 2**-11, (n, scale, inner, worst * 2**11)
        # and the margin the kernels add leaves room for the threshold's own
        # roundings (2^-22 R_I hs and float64 terms)
        assert worst + 2**-22 < 2**-8


def test_bound_is_not_vacuous():
    # the float16 chain does differ from the float32 screen by a visible
    # fraction of the bound on typical data
    rng = np.random.default_rng(51)
    Q = inputs.random_f32(20, 5100)
    worst, _ = _screen_errors(Q, rng)
    assert worst > 0.1 * 2**-11
