"""Benchmark: QUBO states evaluated per second at n=40 on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: one n=40 float32 QUBO, N(0, 1/n) entries with a planted unique
minimiser (seed 2), k=16 lowest states, all 2^40 states enumerated per step.
A step is one full qubo_bf_solve call (plan, table build, persistent Gray-code
walk, merge, float64 rescoring and certificate) with Q resident in HBM.

Prints one JSON line: value = 2^40 * K / elapsed seconds, plus the roofline of
the dominant kernel (the walk) from HIP events recorded around each of its
launches on the call's stream, the same solve with the float32 block screen
(its time, roofline and a bit-identity check against the timed outputs), the CPU oracle timed on a sample of the
same workload, and beside it the paper's own Gray-code method on the host
cores (same sample scheme).  The line also carries the metric's other half:
"batched" (4096 uneven instances in one autotuned, graph-captured launch
sequence against one qubo_bf_solve per instance) and "logz_grad" (768
log-partition forward + adjoint pairs in one call each against one call pair
per (instance, beta)), each with its walk kernels' VALU fractions and an
identity check of the outputs.  Further workloads are reported under "extra"
when --extra is given.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic VALU lane-operations per enumerated state of the block-table walk.
# float32 screen (and the int32 walk): one table addition (v_add_f32 with a DPP
# row broadcast) plus half of a three-input minimum (v_min3_f32 folds two
# states).  Half-precision screen (the float32 default): per block of 64 states
# 32 v_pk_add_f16 (two states each) for C' + Tb, 14 three-input
# v_pk_minimum3_f16 and 2 v_pk_min_f16 for the minimum over b, 2 v_pk_add_f16
# for + Ta, 1 v_pk_minimum3_f16 and 1 v_min_f16 for the minimum over a:
# 52 / 64.  The int16 screen (int32 Q) has no three-input packed minimum:
# 32 v_pk_add_i16, 30 v_pk_min_i16, 2 v_pk_add_i16, 2 minimums: 66 / 64.
ALG_OPS_PER_STATE = 1.5
HALF_OPS_PER_STATE = 52 / 64
INT16_OPS_PER_STATE = 66 / 64
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 3.93e13 non-packed VALU lane-ops/s.
PEAK_LANE_OPS = 256 * 64 * 2.4e9

# HBM bytes per walk launch come from the committed rocprofv3 counter summary
# (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings); they are
# reported only while the walk's sources still hash to the profiled ones.
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "walk_topk_n40_f32_k16_counters.md")
WALK_SOURCES = ("paper_2310_19373_amd/csrc/walk_topk.hip", "paper_2310_19373_amd/csrc/walk.hpp",
                "paper_2310_19373_amd/csrc/wave.hpp", "paper_2310_19373_amd/csrc/common.hpp",
                "paper_2310_19373_amd/csrc/launch.hpp", "paper_2310_19373_amd/build.py")


def walk_sources_sha256() -> str:
    h = hashlib.sha256()
    for rel in WALK_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def committed_traffic():
    """Bytes per walk launch from the counter summary, or None when it is
    missing or was taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    fields = {}
    with open(TRAFFIC_SUMMARY) as f:
        for line in f:
            key, sep, val = line.strip().strip("-* `").partition(":")
            if sep:
                fields[key.strip("` ")] = val.strip(" `")
    if fields.get("kernel_sources_sha256") != walk_sources_sha256():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(Q, n, k):
    import oracle

    rng = np.random.default_rng(123)
    span = 1 << 22
    count = 256  # 256 ranges of 2^22 masks = 2^30 states
    starts = rng.choice(1 << (n - 22), count, replace=False)
    t0 = time.perf_counter()
    for s in starts:
        oracle.topk(Q, k, lo=int(s) << 22, hi=(int(s) << 22) + span)
    dt = time.perf_counter() - t0
    states = count * span
    return {"value": states / dt, "unit": "states/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{count} random prefix ranges of 2^22 masks (2^30 of the 2^40 states), "
                      f"natural-order float64 evaluation, {dt:.1f} s"}


def cpu_paper_method(Q, n):
    """The paper's own method on the host: the Gray-code walk of Algorithm 1
    with the Sec. 3.1 prefix split, float64, O(n) per state, all host cores,
    timed on 256 random 16-bit prefixes of the same instance (2^24 states
    each).  Context beside the oracle baseline, not the target."""
    from oracle import gray_cpu

    m = 16
    rng = np.random.default_rng(124)
    prefixes = rng.choice(1 << m, 256, replace=False)
    gray_cpu.minimum(Q, m, prefixes[:8])  # load the library, touch the pages
    t0 = time.perf_counter()
    gray_cpu.minimum(Q, m, prefixes)
    dt = time.perf_counter() - t0
    states = len(prefixes) * (1 << (n - m))
    return {"value": states / dt, "unit": "states/s", "cores": gray_cpu.max_threads(),
            "kind": "paper's method (Gray-code walk, Algorithm 1 + Sec. 3.1 prefix split, float64)",
            "sample": f"{len(prefixes)} random prefixes of 16 bits, 2^{n - m} states each "
                      f"(2^{int(np.log2(states))} of the 2^40 states), minimum only, {dt:.1f} s",
            # the paper's own CPU figure, quoted: its conclusion brute-forces
            # n=30 in under 4 s on the authors' machine; its timing
            # experiment (Sec. 3) names an Intel Core i7-8700
            "paper_reported": {"value": float(2**30) / 4.0, "unit": "states/s", "bound": "lower",
                               "derivation": "n=30 (2^30 states) in under 4 s",
                               "hardware": "Intel Core i7-8700 (6 cores / 12 threads)",
                               "source": "Conclusion; hardware from the timing experiment of Sec. 3"}}


def _time(fn, reps):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def float_ops_per_state(wide: bool = False):
    """Lane-ops per state of the walk as the library is tuned now: the half
    screen's (float32, float64 and int64 Q, and int32 Q whose inner rows fit
    int16), else the float32 / int32 screen's, or the float64 walk's 3 (a
    64-bit DPP move, v_add_f64, v_min_f64) for wide Q."""
    from paper_2310_19373_amd import _lib

    if _lib.get_tuning(_lib.TUNE_HALF_SCREEN) > 0:
        return HALF_OPS_PER_STATE
    return 3.0 if wide else ALG_OPS_PER_STATE


def int32_ops_per_state():
    """Lane-ops per state of the int32 walk: the int16 screen's when the half
    screens are on (int32 Q whose inner rows fit int16), else the int32
    screen's 1.5."""
    from paper_2310_19373_amd import _lib

    return INT16_OPS_PER_STATE if _lib.get_tuning(_lib.TUNE_HALF_SCREEN) > 0 else ALG_OPS_PER_STATE


def extra_single(dev, name, Q, k, dt, reps, ops_per_state=ALG_OPS_PER_STATE):
    """One full qubo_bf_solve per call on another configuration; states/s of
    the call and the walk kernel's VALU roofline fraction (ops_per_state
    lane-ops per state: 52/64 for the float16 screen, 66/64 for the int16
    screen, 1.5 for the float32 and int32 screens, 3 for the float64 walk's;
    HIP events around the walk launch)."""
    import torch

    from paper_2310_19373_amd import _lib

    n = Q.shape[0]
    Qd = torch.from_numpy(Q).to(dev)
    L = _lib.lib()
    ws_bytes = L.qubo_bf_workspace_size(n, k, dt)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    en = torch.empty(k, dtype=torch.float64 if dt in (_lib.QUBO_F32, _lib.QUBO_F64) else torch.int64, device=dev)
    mk = torch.empty(k, dtype=torch.int64, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream

    def call():
        _lib.check(L.qubo_bf_solve(Qd.data_ptr(), n, n, dt, k, en.data_ptr(), mk.data_ptr(), st.data_ptr(),
                                   ws.data_ptr(), ws_bytes, stream))

    call()
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    _lib.prof_enable(True)
    _lib.prof_collect("walk_topk")
    t = _time(call, reps)
    _lib.prof_enable(False)
    wms, wn = _lib.prof_collect("walk_topk")
    states = float(1 << n)
    walk_s = wms / 1e3 / max(wn, 1)
    return {"workload": name, "states": states, "ms_per_call": t * 1e3, "states_per_s": states / t,
            "walk_ms": walk_s * 1e3, "walk_frac": states * ops_per_state / walk_s / PEAK_LANE_OPS}


def extra_ranges(dev):
    """The n=40 workload cut into 16 prefix ranges (resumable pieces) and
    merged, against one full solve: the cost of chunking a long enumeration."""
    import torch

    from paper_2310_19373_amd import api, inputs

    Q, xstar = inputs.single_n40_f32_planted()
    Qd = torch.from_numpy(Q).to(dev)

    def chunked():
        parts = [api.solve_range(Qd, 16, 4, p, p + 1, check_lower=False) for p in range(16)]
        return api.merge_topk(parts, 16)

    e, m = chunked()
    fe, fm = api.solve(Qd, 16)
    t_chunked = _time(chunked, 2)
    t_full = _time(lambda: api.solve(Qd, 16, check_lower=False), 2)
    states = float(1 << 40)
    return {"workload": "n=40 planted (seed 2), k=16, 16 prefix ranges of 2^36 states + merge",
            "chunked_ms": t_chunked * 1e3, "full_ms": t_full * 1e3, "chunked_states_per_s": states / t_chunked,
            "overhead": t_chunked / t_full - 1.0, "identical_to_full": bool(torch.equal(e, fe) and torch.equal(m, fm))}


def extra_moments(dev):
    """Second moments (marginals on the diagonal) and E_p[f] of the 768
    (instance, beta) pairs: one batched logz_moments call (forward + moment
    walk)."""
    import torch

    from paper_2310_19373_amd import api, inputs

    Q, beta = inputs.logz_256x24()
    Qt = torch.from_numpy(Q).to(dev)
    bt = torch.from_numpy(beta).to(dev)
    api.logz_moments(Qt, bt)
    t = _time(lambda: api.logz_moments(Qt, bt), 3)
    return {"workload": "768 (instance, beta) pairs, n=24 (seed 4): E_p[x_i x_j], E_p[f]",
            "ms": t * 1e3, "states_per_s": 2 * 768 * float(1 << 24) / t}


def extra_sample(dev, nsamples=256):
    """Exact Boltzmann samples of the 768 (instance, beta) pairs, n=24: one
    qubo_logz_sample call (forward enumeration + one wave per sample)."""
    import numpy as np
    import torch

    from paper_2310_19373_amd import api, inputs

    Q, beta = inputs.logz_256x24()
    Qt = torch.from_numpy(Q).to(dev)
    bt = torch.from_numpy(beta).to(dev)
    u = torch.from_numpy(np.random.default_rng(5).random((Q.shape[0], nsamples))).to(dev)
    api.logz_sample(Qt, bt, u)
    t = _time(lambda: api.logz_sample(Qt, bt, u), 3)
    return {"workload": f"768 (instance, beta) pairs, n=24 (seed 4): {nsamples} exact samples each",
            "ms": t * 1e3, "samples_per_s": Q.shape[0] * nsamples / t}


# Algorithmic work per state of the log-partition walks (factored form).
# Forward: on the matrix cores, one multiply-add per state (the product U +=
# B_t^T G_t of step-factor rows and per-lane step weights), 2 flops against
# the float32 matrix peak.  Adjoint (nested form, which every unit of the
# workload takes): the inner sums W go to the matrix cores as in the forward;
# on the VALU, in issue slots of the 4-cycle rate the VALU peak counts, per
# 32 states: the 62 multiply-adds of the nested block sums s and v_a
# (VGPR-only float32 forms, which issue twice as fast: half a slot each), 6
# DPP row broadcasts of the step's factors (one slot each), one reciprocal and
# one exp2 (two slots each).
LOGZ_FWD_FLOPS_PER_STATE = 2
PEAK_MFMA_F32 = 157.3e12  # MI355X dense float32 matrix peak, FLOP/s
LOGZ_BWD_OPS_PER_STATE = (62 / 2 + 6 + 2 + 2) / 32


def leg_batched(dev, plain_loop=True, tune=True):
    """4096 QUBOs, n uniform in [12, 28], k=1: the batched path as a user
    runs it -- a BatchedSolver that autotunes its launch shape on the first
    call and replays a captured HIP graph -- against one qubo_bf_solve call
    per instance, queued on the same stream with no synchronisation between
    calls."""
    import torch

    from paper_2310_19373_amd import _lib, api, inputs

    Q, ns = inputs.batched_4096()
    states = float(sum(1 << int(n) for n in ns))
    t0 = time.perf_counter()
    solver = api.BatchedSolver(len(ns), 28, 1, device=dev, graph=True, autotune=tune)
    solver.load(Q, ns)
    solver.run()  # tunes (first call), captures the graph, replays it
    torch.cuda.synchronize()
    first_call_s = time.perf_counter() - t0
    solver.results()
    t_batched = _time(solver.run, 5)
    e_b, m_b = solver.energies.clone(), solver.masks.clone()
    # the walk kernel's duration: an eager run of the same launch sequence and
    # shape, HIP events around each walk launch
    eager = api.BatchedSolver(len(ns), 28, 1, device=dev, graph=False)
    if solver.setting is not None:
        eager.use_setting(solver.setting)
    eager.load(Q, ns)
    eager.run()
    torch.cuda.synchronize()
    _lib.prof_enable(True)
    _lib.prof_collect("walk_topk")
    _time(eager.run, 3)
    _lib.prof_enable(False)
    wms, wn = _lib.prof_collect("walk_topk")
    walk_s = wms / 1e3 / max(wn, 1)
    out = {"workload": "4096 QUBOs, n uniform in [12,28] (seed 3), float32 N(0,1), k=1",
           "states": states, "batched_ms": t_batched * 1e3, "batched_states_per_s": states / t_batched,
           "kernel": "walk_topk_h16_kernel", "walk_ms": walk_s * 1e3,
           "walk_frac": states * HALF_OPS_PER_STATE / walk_s / PEAK_LANE_OPS,
           "first_call_s": first_call_s, "launch_shape": solver.setting,
           "untuned_ms": solver.tune_result.start_ms if solver.tune_result else None}
    if plain_loop:
        L = _lib.lib()
        Qs = [torch.from_numpy(np.ascontiguousarray(Q[b, :int(n), :int(n)])).to(dev) for b, n in enumerate(ns)]
        ws_bytes = max(L.qubo_bf_workspace_size(int(n), 1, _lib.QUBO_F32) for n in ns)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        en = torch.empty((len(ns), 1), dtype=torch.float64, device=dev)
        mk = torch.empty((len(ns), 1), dtype=torch.int64, device=dev)
        st = torch.empty(len(ns), dtype=torch.int32, device=dev)
        stream = torch.cuda.current_stream(dev).cuda_stream

        def plain():
            for b, n in enumerate(ns):
                _lib.check(L.qubo_bf_solve(Qs[b].data_ptr(), int(n), int(n), _lib.QUBO_F32, 1, en[b].data_ptr(),
                                           mk[b].data_ptr(), st[b:b + 1].data_ptr(), ws.data_ptr(), ws_bytes,
                                           stream))

        plain()
        t_plain = _time(plain, 1)
        out.update({"plain_ms": t_plain * 1e3, "speedup_vs_plain": t_plain / t_batched,
                    "identical_to_plain": bool(torch.equal(en, e_b) and torch.equal(mk, m_b)
                                               and not bool(st.any()))})
    return out


def leg_logz(dev, plain_loop=True):
    """768 (instance, beta) pairs, 256 QUBOs n=24 x beta in {0.5, 1, 4}: one
    batched qubo_logz_fwd + qubo_logz_bwd call pair against one fwd + bwd call
    pair per (instance, beta), all through the C ABI, queued on one stream
    with no synchronisation between calls."""
    import torch

    from paper_2310_19373_amd import _lib, inputs

    Q, beta = inputs.logz_256x24()
    P, n = len(beta), Q.shape[1]
    L = _lib.lib()
    stream = torch.cuda.current_stream(dev).cuda_stream
    Qt = torch.from_numpy(Q).to(dev)
    bt = torch.from_numpy(beta).to(dev)
    ns = torch.full((P,), n, dtype=torch.int32, device=dev)
    gl = torch.ones(P, dtype=torch.float32, device=dev)

    def buffers(batch):
        nbytes = L.qubo_logz_workspace_size(batch, n)
        return {"ws": torch.empty(nbytes, dtype=torch.uint8, device=dev), "nbytes": nbytes,
                "lz": torch.empty(P, dtype=torch.float64, device=dev), "st": torch.empty(P, dtype=torch.int32, device=dev),
                "gq": torch.empty_like(Qt), "gb": torch.empty(P, dtype=torch.float32, device=dev)}

    def fwd_bwd(B, p, cnt):
        q, b = Qt[p].data_ptr(), bt[p].data_ptr()
        lz, st = B["lz"][p].data_ptr(), B["st"][p].data_ptr()
        _lib.check(L.qubo_logz_fwd(cnt, q, n, ns[p].data_ptr(), b, lz, st, B["ws"].data_ptr(), B["nbytes"], stream))
        _lib.check(L.qubo_logz_bwd(cnt, q, n, ns[p].data_ptr(), b, lz, gl[p].data_ptr(), B["gq"][p].data_ptr(),
                                   B["gb"][p].data_ptr(), st, B["ws"].data_ptr(), B["nbytes"], stream))

    Bb = buffers(P)
    fwd_bwd(Bb, 0, P)
    torch.cuda.synchronize()
    assert not bool(Bb["st"].any())
    _lib.prof_enable(True)
    for nm in ("walk_exp", "walk_grad"):
        _lib.prof_collect(nm)
    t_batched = _time(lambda: fwd_bwd(Bb, 0, P), 5)
    _lib.prof_enable(False)
    kern = {nm: _lib.prof_collect(nm) for nm in ("walk_exp", "walk_grad")}
    states = float(P) * (1 << n)
    fwd_s = kern["walk_exp"][0] / 1e3 / max(kern["walk_exp"][1], 1)
    bwd_s = kern["walk_grad"][0] / 1e3 / max(kern["walk_grad"][1], 1)
    out = {"workload": "768 (instance, beta) pairs: 256 QUBOs n=24 float32 N(0,1/n) (seed 4) x beta {0.5,1,4}",
           "states_per_pass": states, "batched_fwd_bwd_ms": t_batched * 1e3,
           "kernels": {"walk_exp_fac_kernel": {"ms": fwd_s * 1e3, "bound": "mfma",
                                               "flops_per_state": LOGZ_FWD_FLOPS_PER_STATE,
                                               "frac": states * LOGZ_FWD_FLOPS_PER_STATE / fwd_s / PEAK_MFMA_F32},
                       "walk_grad_fac_kernel": {"ms": bwd_s * 1e3, "ops_per_state": LOGZ_BWD_OPS_PER_STATE,
                                                "frac": states * LOGZ_BWD_OPS_PER_STATE / bwd_s / PEAK_LANE_OPS}}}
    if plain_loop:
        Bp = buffers(1)

        def plain():
            for p in range(P):
                fwd_bwd(Bp, p, 1)

        plain()
        t_plain = _time(plain, 1)
        gd = (Bp["gq"] - Bb["gq"]).abs().max().item() / max(Bb["gq"].abs().max().item(), 1e-30)
        out.update({"plain_fwd_bwd_ms": t_plain * 1e3, "speedup_vs_plain": t_plain / t_batched,
                    "identical_logz": bool(torch.equal(Bp["lz"], Bb["lz"])),
                    "identical_grad": bool(torch.equal(Bp["gq"], Bb["gq"]) and torch.equal(Bp["gb"], Bb["gb"])),
                    "grad_max_rel_diff": gd, "status_ok": not bool(Bp["st"].any() or Bb["st"].any())})
    return out


def valu_rates():
    """Cycles per wave64 VALU instruction per SIMD for each instruction form of
    the walks (the probe library built beside the solver; the shader clock is
    read in the same launch).  One JSON line per form and occupancy."""
    import ctypes

    path = os.path.join(ROOT, "paper_2310_19373_amd", "libvalu_rates.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    P = ctypes.CDLL(path)
    P.valu_rate.restype = ctypes.c_int
    P.valu_rate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_float),
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    P.valu_rate_form_name.restype = ctypes.c_char_p
    for wps in (2, 4, 8):
        for form in range(P.valu_rate_forms()):
            ms, mhz, cyc = ctypes.c_float(), ctypes.c_double(), ctypes.c_double()
            rc = P.valu_rate(form, wps, 20000, ctypes.byref(ms), ctypes.byref(mhz), ctypes.byref(cyc))
            if rc != 0:
                raise RuntimeError(f"valu_rate({form}, {wps}) returned {rc}")
            print(json.dumps({"form": P.valu_rate_form_name(form).decode(), "waves_per_simd": wps,
                              "ms": round(ms.value, 4), "shader_mhz": round(mhz.value, 1),
                              "cycles_per_instr": round(cyc.value, 3)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extra", action="store_true",
                    help="also time further workloads (n=20, n=32 int32, n=40 float64, ranges, moments, samples)")
    ap.add_argument("--only", choices=("n40", "batched", "logz", "n40_f64", "n32_i32"),
                    help="n40: the headline n=40 solve (and its float32-screen repeat) alone, the line "
                         "without the batched / logZ legs and host baselines, for profiling; otherwise "
                         "run only that secondary workload, without the one-call-per-instance loop")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched leg: keep the current launch shape (knobs or QUBO_BF_* variables) untuned")
    ap.add_argument("--sources-sha", action="store_true", help="print the walk sources' sha256 and exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (counter calibration for HBM bytes)")
    ap.add_argument("--valu-rates", action="store_true",
                    help="run only the VALU issue-cost probe: cycles per wave64 instruction of each form the "
                         "walks use, at 4 and 8 waves per SIMD")
    args = ap.parse_args()
    if args.sources_sha:
        print(walk_sources_sha256())
        return
    if args.valu_rates:
        valu_rates()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library runs on one device; "
              "across GPUs the enumeration would shard its work units by their top prefix bits", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2310_19373_amd import _lib, api, inputs

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "launches": 3}), flush=True)
        return
    if args.only and args.only != "n40":
        if args.only == "batched":
            res = leg_batched(dev, plain_loop=False, tune=not args.no_tune)
        elif args.only == "n32_i32":
            res = extra_single(dev, "n=32 int32 uniform [-100,100] (seed 1), k=16", inputs.single_n32_i32(), 16,
                               _lib.QUBO_I32, 10, ops_per_state=int32_ops_per_state())
        elif args.only == "n40_f64":
            res = extra_single(dev, "n=40 planted (seed 2) as float64 Q, k=16",
                               inputs.single_n40_f32_planted()[0].astype("float64"), 16, _lib.QUBO_F64, 3,
                               ops_per_state=float_ops_per_state(wide=True))
        else:
            res = leg_logz(dev, plain_loop=False)
        print(json.dumps({args.only: res}), flush=True)
        return
    Q, xstar = inputs.single_n40_f32_planted()
    n, k = 40, 16
    Qd = torch.from_numpy(Q).to(dev)
    L = _lib.lib()
    ws_bytes = L.qubo_bf_workspace_size(n, k, _lib.QUBO_F32)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    en = torch.empty(k, dtype=torch.float64, device=dev)
    masks = torch.empty(k, dtype=torch.int64, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream

    def step():
        _lib.check(L.qubo_bf_solve(Qd.data_ptr(), n, n, _lib.QUBO_F32, k, en.data_ptr(), masks.data_ptr(),
                                   status.data_ptr(), ws.data_ptr(), ws_bytes, stream))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert int(status.item()) == 0, f"status {int(status.item())}"
    assert int(masks[0].item()) == xstar, "planted minimiser not found"

    _lib.prof_enable(True)
    _lib.prof_collect("walk_topk")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    _lib.prof_enable(False)
    walk_ms, walk_n = _lib.prof_collect("walk_topk")
    assert int(status.item()) == 0 and int(masks[0].item()) == xstar

    states = float(1 << n)
    value = states * args.steps / elapsed
    walk_avg_s = walk_ms / 1e3 / max(walk_n, 1)
    ops = float_ops_per_state()
    achieved = states * ops / walk_avg_s / 1e12
    peak = PEAK_LANE_OPS / 1e12
    out = {
        "metric": "QUBO states evaluated/sec at n=40",
        "value": value,
        "unit": "states/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f16+f64" if ops == HALF_OPS_PER_STATE else "f32",
        "data": "synthetic",
        "config": {"workload": "single QUBO n=40, float32 N(0,1/n) + planted minimiser (seed 2), k=16, "
                               "2^40 states per step, float64 rescoring of the top candidates",
                   "screen": ("packed float16 block screen with a margin that keeps every block a float32 "
                              "screen keeps; passing blocks replayed in float64; results identical to the "
                              "float32 walk") if ops == HALF_OPS_PER_STATE else "float32 block screen"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "T VALU lane-op/s",
                     "frac": achieved / peak, "traffic": committed_traffic(),
                     "kernel": "walk_topk_h16_kernel" if ops == HALF_OPS_PER_STATE else "walk_topk_kernel",
                     "kernel_ms": walk_avg_s * 1e3,
                     "ops_per_state": ops},
    }
    if ops == HALF_OPS_PER_STATE:
        # the same solve with the float32 block screen, untimed in `value`:
        # its own roofline and a check that the outputs are bit-identical
        ref_e, ref_m = en.clone(), masks.clone()
        saved = _lib.get_tuning(_lib.TUNE_HALF_SCREEN)
        _lib.set_tuning(_lib.TUNE_HALF_SCREEN, -1)
        try:
            if L.qubo_bf_workspace_size(n, k, _lib.QUBO_F32) > ws_bytes:  # the plan may differ
                ws_bytes = L.qubo_bf_workspace_size(n, k, _lib.QUBO_F32)
                ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
            step()
            torch.cuda.synchronize()
            reps = max(1, min(args.steps, 5))
            _lib.prof_enable(True)
            _lib.prof_collect("walk_topk")
            t1 = time.perf_counter()
            for _ in range(reps):
                step()
            torch.cuda.synchronize()
            el32 = time.perf_counter() - t1
            _lib.prof_enable(False)
            w32_ms, w32_n = _lib.prof_collect("walk_topk")
        finally:
            _lib.set_tuning(_lib.TUNE_HALF_SCREEN, saved)
        w32_s = w32_ms / 1e3 / max(w32_n, 1)
        out["float32_screen"] = {
            "value": states * reps / el32, "ms_per_step": el32 * 1e3 / reps, "steps": reps,
            "kernel": "walk_topk_kernel", "kernel_ms": w32_s * 1e3, "ops_per_state": ALG_OPS_PER_STATE,
            "frac": states * ALG_OPS_PER_STATE / w32_s / PEAK_LANE_OPS,
            "identical": bool(torch.equal(ref_e, en) and torch.equal(ref_m, masks) and int(status.item()) == 0)}
    if args.only == "n40":
        print(json.dumps(out), flush=True)
        return
    # the other half of the metric: batched solves and logZ gradients against
    # one-at-a-time launches of the same library calls
    out["batched"] = leg_batched(dev, tune=not args.no_tune)
    out["logz_grad"] = leg_logz(dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(Q, n, k)
        out["cpu_paper_method"] = cpu_paper_method(Q, n)
    if args.extra:
        out["extra"] = {
            "single_n20_f32": extra_single(dev, "n=20 float32 N(0,1) (seed 0), k=8", inputs.single_n20_f32(), 8,
                                           _lib.QUBO_F32, 50, ops_per_state=float_ops_per_state()),
            "single_n32_i32": extra_single(dev, "n=32 int32 uniform [-100,100] (seed 1), k=16",
                                           inputs.single_n32_i32(), 16, _lib.QUBO_I32, 10,
                                           ops_per_state=int32_ops_per_state()),
            "single_n40_f64": extra_single(dev, "n=40 planted (seed 2) as float64 Q, k=16",
                                           inputs.single_n40_f32_planted()[0].astype("float64"), 16, _lib.QUBO_F64,
                                           3, ops_per_state=float_ops_per_state(wide=True)),
            "ranges": extra_ranges(dev),
            "moments": extra_moments(dev), "sample": extra_sample(dev)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
