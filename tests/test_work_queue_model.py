"""CPU model of the walks' work distribution (the planner's queue set-up in
setup.hip plan_kernel and WorkIter in walk.hpp), checking the design: every
work unit is walked exactly once and each wave's units increase (the
flush-once-per-instance rule relies on it), for grids larger and smaller than
the unit count and every chunk cap, under random interleavings of the waves.

The model restates the integer arithmetic of those two pieces of device code
(segment bounds, static first runs, guided pull sizes, the look-before-pull
rule near a segment's end); the GPU parity tests check the kernels
themselves.
"""
import random

import pytest

K = 8      # queue segments (one per XCD)
WPB = 4    # waves per workgroup


def plan(tu, waves, chunk_cap):
    c = max(1, min(tu // (max(waves, 1) * 4), chunk_cap))
    blocks = waves // WPB
    seg = []
    for x in range(K):
        b0, b1 = tu * x // K, tu * (x + 1) // K
        wx = ((blocks - x + K - 1) // K) * WPB if blocks > x else 0
        seg.append([min(b0 + wx * c, b1), b1])
    return c, seg


class Wave:
    def __init__(self, bi, wv, cap, seg):
        self.bi, self.wv, self.sg = bi, wv, bi % K
        self.seg_end = seg[self.sg][1]
        self.first, self.want, self.left = True, cap, None
        self.u = self.u_end = 0
        self.last = -1


def step(w, tu, blocks, cap, waves2, seg):
    if w.u < w.u_end:
        w.u += 1
        return w.u - 1
    if w.first:
        w.first = False
        x = w.sg
        b0 = tu * x // K
        wx = ((blocks - x + K - 1) // K) * WPB if blocks > x else 0
        w.left = w.seg_end - min(b0 + wx * cap, w.seg_end)
        c = b0 + ((w.bi // K) * WPB + w.wv) * cap
        if c < w.seg_end:
            w.u, w.u_end = c + 1, min(c + cap, w.seg_end)
            return c
    while True:
        if w.left is not None and w.left <= waves2 * cap:
            avail = [s for s in range(K) if s >= w.sg and seg[s][0] < seg[s][1]]
            if not avail:
                return None
            if avail[0] != w.sg:
                w.sg, w.seg_end, w.want = avail[0], seg[avail[0]][1], cap
            w.left = None
        c = seg[w.sg][0]
        seg[w.sg][0] += w.want
        if c < w.seg_end:
            w.u, w.u_end = c + 1, min(c + w.want, w.seg_end)
            w.left = w.seg_end - w.u_end
            share = w.left // waves2
            w.want = 1 if share < 1 else min(share, cap)
            return c
        w.left = 0


@pytest.mark.parametrize("tu,waves", [(1, 4), (3, 4), (7, 12), (100, 64), (2048, 2048), (4096, 3072), (4095, 3072),
                                      (65536, 4096), (16384, 4096), (1000, 4096), (12345, 3072), (5, 4096), (9, 4)])
@pytest.mark.parametrize("chunk_cap", [1, 2, 8])
def test_every_unit_once_and_increasing_per_wave(tu, waves, chunk_cap):
    for seed in range(3):
        rnd = random.Random(seed)
        cap, seg = plan(tu, waves, chunk_cap)
        blocks = waves // WPB
        waves2 = 2 * max(waves // K, 1)
        ws = [Wave(bi, wv, cap, seg) for bi in range(blocks) for wv in range(WPB)]
        taken = [0] * tu
        active = list(ws)
        while active:
            w = rnd.choice(active)
            u = step(w, tu, blocks, cap, waves2, seg)
            if u is None:
                active.remove(w)
                continue
            assert u > w.last
            w.last = u
            taken[u] += 1
        assert taken == [1] * tu
