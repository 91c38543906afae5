// Persistent top-k enumeration kernel (the hot path).
//
// Each wave pulls work units from a queue.  A unit fixes the tile bits; lane l
// fixes the lane bits (the prefix split of Sec. 3.1: 2^(L+tb) independent
// sub-walks whose results are min-combined).  Per lane and unit:
//
//   * lane init: E_P, the per-lane inner table C'(j) = E_I(j) + X_PI(p, j)
//     (64 entries of float32 or int32, or 32 of float64, in VGPRs) and the
//     per-lane cross fields
//     c_l = sum_{v in prefix} S_{l v} x_v of the outer bits (LDS);
//   * outer walk over t = 0 .. 2^no - 1 in reflected Gray order: step t flips
//     bit l = CTZ(t) (Sec. 2.2), turning it on iff bit l+1 of t is 0; the
//     per-lane scalar KE = E_P + X_PO + E_O moves by +-c_l plus the uniform
//     E_O(g(t)) (the single-flip update of Eq. 2, Sec. 2.1, restricted to the prefix/outer cross terms);
//   * 64 inner states per step: e_j = C'(j) + T'(g(t); j).  The default
//     screens them in packed float16 (int16 for int32 Q) with T' split into
//     two scalar-register tables (walk_unit_h16 / walk_unit_i16 below, about
//     one packed instruction per state); the float32 / int32 screen
//     broadcasts T' across each 16-lane row by DPP (one v_add_*_dpp per state)
//     and folds by v_min3 (half an instruction per state); the float64 walk
//     takes 32 inner states per step at three instructions per state
//     (v_mov_b64_dpp, v_add_f64, v_min_f64);
//   * if the block minimum can beat the wave's threshold (rare after warm-up),
//     the block is replayed with exact float64 / int64 keys and the candidates
//     are inserted into the wave's sorted top-K' list (lexicographic (energy,
//     mask) order, ties to the lower mask).
//
// Thresholds: a wave discards a block only if min_j e_j + KE exceeds its
// threshold thr = min(K'-th key of its own list, the instance's published
// threshold, an a-priori bound).  Every threshold is backed by K' real states,
// so discarded states cannot enter the final top-K' (float: up to the bound
// eps on the float32 rounding of e_j, which the certificate accounts for).
#include "walk.hpp"

namespace qbf {

namespace {

// Writes the wave's list to the next free slot of instance b.  A count above
// the slot capacity is reported by the finalize kernel (it cannot happen: a
// wave flushes an instance at most once per contiguous run of its units).
//
// A list whose best entry lies above the instance's published threshold is
// dropped: the threshold only decreases and is backed by K' real states, so
// each of the instance's K' best states has a key at most the final
// threshold and sits, by then, in the list of the wave that walked it --
// whose best entry is therefore at most the threshold, and that list is
// flushed.  Dropping the others spares one slot-counter atomic per wave per
// instance (thousands on one address for a single instance).
__device__ void flush(const Views& v, int b, double lkey, uint64_t lmask, int lane) {
  if (!(readlane_f64(lkey, 0) <= load_gthr(v, b))) return;  // uniform
  const InstU I = load_inst(v, b);
  const uint32_t slot = (uint32_t)uniform_i32((int)atomicAdd(v.flushcnt + b, lane == 0 ? 1u : 0u));
  if ((int64_t)slot < I.slot_cap && lane < I.kp) {
    const gptr<Slot> d = gp(v.slots) + (I.slot_off + slot) * I.kp + lane;
    d->key = lkey;
    d->mask = lmask;
  }
}

// Replay of one outer step with exact keys; inserts every state whose key does
// not exceed thr into the list.  Uniform control flow, all lanes active.
template <class E>
__device__ __forceinline__ void replay(const Views& v, int b, const InstU& I, uint32_t t, uint64_t p, bool valid,
                                       typename Ar<E>::W KE, double& thr, double& lkey, uint64_t& lmask,
                                       uint64_t& pub, const typename Ar<E>::W* myc, int lane) {
  using W = typename Ar<E>::W;
  const int pos0 = I.B + I.no;
  const gptr<const W> ei = gp((const W*)v.ei) + (int64_t)b * 64;
  W cI[6];
#pragma unroll
  for (int u = 0; u < 6; ++u) cI[u] = myc[(kCIRow + u) * kWave + lane];  // written by lane_init
  const gptr<const StepRec> r = gp((const StepRec*)v.rec) + I.tab_off + t;
  W h[6];
#pragma unroll
  for (int u = 0; u < 6; ++u) h[u] = (W)r->h[u];
  const uint64_t base = valid ? ((p << pos0) | (gray((uint64_t)t) << I.B)) : 0;
  for (int j = 0; j < (1 << I.B); ++j) {
    W cj = ei[j], tj = 0;
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      if ((j >> u) & 1) {
        cj += cI[u];
        tj += h[u];
      }
    }
    const double key = (double)(KE + cj + tj);
    uint64_t bal = ballot(valid && key <= thr);
    while (bal) {
      const int src = __builtin_ctzll(bal);
      bal &= bal - 1;
      const double ck = readlane_f64(key, src);
      if (ck <= thr) {
        const uint64_t cm = readlane_u64(base, src) | (uint64_t)j;
        if (list_insert(lkey, lmask, ck, cm, I.kp, lane)) {
          const double lt = readlane_f64(lkey, I.kp - 1);
          if (lt < thr) thr = lt;
        }
      }
    }
  }
  const double lt = readlane_f64(lkey, I.kp - 1);
  if (lt < __builtin_inf()) {
    const uint64_t e = enc_key(lt);
    if (e < pub) {
      if (lane == 0) atomicMin((unsigned long long*)(v.gthr + b), (unsigned long long)e);
      pub = e;
    }
  }
}

template <class E>
__device__ __forceinline__ void walk_unit(const Views& v, int b, const InstU& I, uint64_t local, double& lkey,
                                          uint64_t& lmask, uint64_t& pub, typename Ar<E>::W* myc, int lane) {
  using W = typename Ar<E>::W;
  using V = typename Ar<E>::V;
  constexpr int NB = Ar<E>::NB;
  constexpr bool kInt = std::is_same_v<E, int32_t>;
  const bool valid = lane < (1 << I.L);
  const uint64_t p = (local << I.L) | (uint64_t)lane;

  // ---- lane init: prefix energy, inner table, outer cross fields
  E C[NB];
  const W EP = lane_init<E, NB>(v, b, I, local, valid, myc, lane, C);

  // ---- outer walk
  // Dp = thr - E_P - X_PO(p, g(t)) is kept instead of the running value itself:
  // the filter of step t is  min_j e_j <= Dp - E_O(g(t)).  A threshold change by
  // delta moves Dp by delta.
  using Acc = std::conditional_t<kInt, int32_t, double>;
  // pub also tracks the lowest threshold seen, so a wave publishes (one
  // atomic) only a value below what the instance already has
  const double g0 = load_gthr(v, b);
  if (enc_key(g0) < pub) pub = enc_key(g0);
  double thr = fmin(fmin(g0, I.big), readlane_f64(lkey, I.kp - 1));
  Acc Dp = kInt ? (Acc)((int32_t)thr - (int32_t)EP) : (Acc)(thr - (double)EP);
  const uint32_t steps = 1u << I.no;
  // T' rows through a buffer resource: per-lane byte offset in a VGPR (fixed),
  // per-step row offset in an SGPR, no address arithmetic on the VALU; reads
  // past the instance's rows return zeros.
  const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(gp((const E*)v.tab) + I.tab_off * NB), (short)0, (int)(steps * (uint32_t)(NB * sizeof(E))),
      0x00020000);
  const int qoff = (lane & 15) * 16;
  const gptr<const double> eod = gp((const double*)v.eod) + I.tab_off;
  const gptr<const int32_t> eoi = gp((const int32_t*)v.eoi) + I.tab_off;
  const W c0 = I.no > 0 ? myc[lane] : (W)0;
  const W c1 = I.no > 1 ? myc[kWave + lane] : (W)0;
  const W c2 = I.no > 2 ? myc[2 * kWave + lane] : (W)0;

  // Operands of a step (T' row in the row-broadcast layout, E_O term), loaded
  // one step ahead; the index is clamped so loads are unconditional.
  struct Ops {
    V tv;
    Acc eo;  // +E_O (float path) or -E_O (int path)
  };
  auto load = [&](uint32_t t) {
    const uint32_t tt = t < steps ? t : steps - 1;
    Ops o;
    o.tv = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(
                                     trs, qoff, (int)(tt * (uint32_t)(NB * sizeof(E))), 0));
    if constexpr (kInt) o.eo = eoi[tt];
    else o.eo = eod[tt];
    return o;
  };
  // Threshold refresh: fold an improvement of thr into Dp.
  auto retune = [&](double nthr) {
    if constexpr (kInt) Dp += (int32_t)nthr - (int32_t)thr;
    else Dp += nthr - thr;
    thr = nthr;
  };
  // Block minimum over the 64 inner states of step t and the filter.
  auto body = [&](uint32_t t, const Ops& o) {
    E acc = Ar<E>::inv();
    if constexpr (std::is_same_v<E, double>) {
      block_min_f64<0>(acc, o.tv.x, C);
      block_min_f64<1>(acc, o.tv.y, C);
    } else {
      block_min<0, 0>(acc, o.tv.x, C);
      block_min<1, 0>(acc, o.tv.y, C);
      block_min<2, 0>(acc, o.tv.z, C);
      block_min<3, 0>(acc, o.tv.w, C);
    }
    bool hit;
    if constexpr (kInt) hit = acc <= Dp + o.eo;
    else hit = (double)acc <= Dp - o.eo;
    if (__builtin_expect(ballot(hit) != 0, 0)) {
      double nthr = thr;
      W KE;
      if constexpr (kInt) KE = (int64_t)(int32_t)thr - (int64_t)Dp - (int64_t)o.eo;
      else KE = thr - Dp + o.eo;
      replay<E>(v, b, I, t, p, valid, KE, nthr, lkey, lmask, pub, myc, lane);
      retune(nthr);
    }
  };
  // Flip of a bit into step t: it turns on (Dp -= c) or off (Dp += c).
  auto flip_on = [&](W c) { Dp -= (Acc)c; };
  auto flip_off = [&](W c) { Dp += (Acc)c; };
  auto flip_sign = [&](bool off, W c) {  // sign known only at run time (uniform)
    if constexpr (kInt) {
      if (off) flip_off(c);
      else flip_on(c);
    } else {
      Dp = __builtin_fma(off ? 1.0 : -1.0, c, Dp);
    }
  };
  auto flip = [&](uint32_t t) {  // general flip: bit CTZ(t), off iff bit CTZ(t)+1 of t is set
    const int l = __builtin_ctz(t);
    flip_sign((t >> (l + 1)) & 1, myc[l * kWave + lane]);
  };

  if (steps < 16) {
    // short walks (small instances): one step at a time
    Ops o = load(0);
    for (uint32_t t = 0; t < steps; ++t) {
      const Ops on = load(t + 1);
      if (t) flip(t);
      body(t, o);
      o = on;
    }
    return;
  }
  // steps >= 16: unrolled by 8.  Within group q (t = 8q .. 8q+8) bit 0 flips
  // on at 8q+1 and 8q+5 and off at 8q+3 and 8q+7, bit 1 on at 8q+2 and off at
  // 8q+6, bit 2 at 8q+4 (off for odd q), bit 3+CTZ(q+1) at 8q+8.
  Ops ev = load(0), od = load(1);
  body(0, ev);
  ev = load(2);
  const uint32_t groups = steps >> 3;
  for (uint32_t q = 0;; ++q) {
    const uint32_t t = 8 * q;
    flip_on(c0);
    body(t + 1, od);
    od = load(t + 3);
    flip_on(c1);
    body(t + 2, ev);
    ev = load(t + 4);
    flip_off(c0);
    body(t + 3, od);
    od = load(t + 5);
    flip_sign(q & 1, c2);
    body(t + 4, ev);
    ev = load(t + 6);
    flip_on(c0);
    body(t + 5, od);
    od = load(t + 7);
    flip_off(c1);
    body(t + 6, ev);
    ev = load(t + 8);
    flip_off(c0);
    body(t + 7, od);
    od = load(t + 9);
    if (q + 1 == groups) break;
    flip(t + 8);
    body(t + 8, ev);
    ev = load(t + 10);
    if (((q + 1) & 7) == 0) {
      const double g = load_gthr(v, b);
      if (enc_key(g) < pub) pub = enc_key(g);
      if (g < thr) retune(g);
    }
  }
}

// ---- the walk with the half-precision screen (float32, float64, int64 Q) ---
//
// Same walk, same replay, same thresholds; only the per-step block screen
// changes.  The inner index j = b | a << 4 splits 4 + 2 and T'(g(t); j) =
// Tb(b) + Ta(a) (T' is linear in the inner bits), so one step reads a 64-byte
// HalfRow with scalar loads and computes, in packed float16 on the scaled
// values,
//   m = min_a [ Ta(a) + min_b (C'(b | a << 4) + Tb(b)) ]
// with C' paired as (a, a + 2) per register: 32 v_pk_add_f16 (two states
// each, Tb(b) taken from either half of a scalar register by op_sel), 16
// three-input v_pk_minimum3_f16 and 2 v_pk_min_f16 folding each 16-register
// group, 2 v_pk_add_f16 for + Ta and 2 final minimums: 52 instructions for 64
// states.  The operands are finite or +inf (every scaled table value is below
// 2^13 in magnitude, unused states are +inf), so no NaN reaches the IEEE
// minimum and it selects the same value as the ordinary minimum.  The float64
// offset Dp is kept scaled by hscale (exact: a power of two), and the block
// passes when m <= Dp - tau, tau = hscale E_O - hmargin.  hmargin makes the
// half screen pass every block the float32 (or float64) screen passes; the
// replay recomputes passing blocks with exact keys.
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(4))) uint32_t* half_words_t;

__device__ __forceinline__ h2 as_h2(uint32_t x) { return __builtin_bit_cast(h2, x); }
__device__ __forceinline__ h2 hmin2(h2 a, h2 b) { return __builtin_elementwise_min(a, b); }
// one v_pk_minimum3_f16
__device__ __forceinline__ h2 hmin3(h2 a, h2 b, h2 c) {
  return __builtin_elementwise_minimum(__builtin_elementwise_minimum(a, b), c);
}
__device__ __forceinline__ h2 hswap(h2 x) { return __builtin_shufflevector(x, x, 1, 0); }

__device__ __forceinline__ float half_block_min(const HalfRow& r, const h2 (&C)[2][16]) {
  h2 m[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    h2 s[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const h2 x = as_h2(r.tb[c >> 1]);
      s[c] = C[a][c] + ((c & 1) ? __builtin_shufflevector(x, x, 1, 1) : __builtin_shufflevector(x, x, 0, 0));
    }
    // 16 -> 6 -> 2 -> 1
    h2 t[6];
#pragma unroll
    for (int i = 0; i < 5; ++i) t[i] = hmin3(s[3 * i], s[3 * i + 1], s[3 * i + 2]);
    t[5] = s[15];
    m[a] = hmin2(hmin3(t[0], t[1], t[2]), hmin3(t[3], t[4], t[5])) + as_h2(r.ta[a]);
  }
  // x.x = min(m0.x, m1.x, m1.y), x.y = min(m0.y, m1.y, m1.x): together all four
  const h2 x = hmin3(m[0], m[1], hswap(m[1]));
  return (float)hmin2(x, hswap(x)).x;
}

// Waits for every scalar-memory / LDS result in flight (the row of the step
// about to run); issued before the next row's loads so that wait never covers
// them.
__device__ __forceinline__ void wait_rows() {
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_sched_barrier(0);
}

// kRowStride: HalfRow units between consecutive step rows (1: the float
// layout; kInt16RowStride: an int32 instance beyond the int32 walk's range,
// whose rows sit in the int32 layout's 256-byte step slots).
// Issue priority by progress through the unit, for launches with about one
// unit per wave: a SIMD issues from the ready wave of highest priority (then
// the oldest), so without this the waves sharing it finish their units one
// after another and the last ones run alone, at one wave's issue rate.  A
// wave that is ahead yields to those behind it: priority 3 in the first
// quarter of its steps, down to 0 in the last.
__device__ __forceinline__ void pace(uint32_t done, uint32_t total) {
  const uint32_t quarter = (4 * done) / total;
  if (quarter == 0) __builtin_amdgcn_s_setprio(3);
  else if (quarter == 1) __builtin_amdgcn_s_setprio(2);
  else if (quarter == 2) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
}

template <int kRowStride = 1>
__device__ __forceinline__ void walk_unit_h16(const Views& v, int b, const InstU& I, uint64_t local, double& lkey,
                                              uint64_t& lmask, uint64_t& pub, double* myc, int lane,
                                              bool paced = false) {
  const bool valid = lane < (1 << I.L);
  const uint64_t p = (local << I.L) | (uint64_t)lane;
  const double hs = uniform_f64(gp((const Inst*)v.inst)[b].hscale);
  const double his = 1.0 / hs;  // exact: hs is a power of two

  // C'(j), j = c | a << 4, as float16 pairs (a, a + 2) of C' * hs: float32
  // rounding, an exact float32 scaling (|C' hs| < 2^13), one float16 rounding
  int hexp;
  frexp(hs, &hexp);
  hexp -= 1;  // hs = 2^hexp
  h2 C16[2][16];
  const double g0 = load_gthr(v, b);  // issued first: its latency overlaps the set-up's
  const double EP = lane_init_with<float, 64, true>(v, b, I, local, valid, myc, lane, [&](int j, bool ok, double cj) {
    const float f = ok ? (float)cj : __builtin_inff();
    C16[(j >> 4) & 1][j & 15][j >> 5] = (_Float16)__builtin_ldexpf(f, hexp);
  });

  if (enc_key(g0) < pub) pub = enc_key(g0);
  double thr = fmin(fmin(g0, I.big), readlane_f64(lkey, I.kp - 1));
  double Dp = (thr - EP) * hs;  // the float32 walk's Dp, scaled
  const uint32_t steps = 1u << I.no;
  // the rows through the constant address space: scalar loads
  const half_words_t rows = (half_words_t)((const HalfRow*)v.tab + I.tab_off * kRowStride);
  const double c0 = I.no > 0 ? myc[lane] * hs : 0.0;
  const double c1 = I.no > 1 ? myc[kWave + lane] * hs : 0.0;
  const double c2 = I.no > 2 ? myc[2 * kWave + lane] * hs : 0.0;

  auto row = [&](uint32_t t) -> HalfRow {
    const half_words_t w = rows + (size_t)(t < steps ? t : steps - 1) * (kRowStride * sizeof(HalfRow) / 4);
    HalfRow r;
#pragma unroll
    for (int c = 0; c < 8; ++c) r.tb[c] = w[c];
    r.ta[0] = w[8];
    r.ta[1] = w[9];
    r.tau = __builtin_bit_cast(double, (uint64_t)w[12] | ((uint64_t)w[13] << 32));
    return r;
  };
  auto retune = [&](double nthr) {
    Dp += (nthr - thr) * hs;
    thr = nthr;
  };
  auto body = [&](uint32_t t, const HalfRow& r) {
    const float m = half_block_min(r, C16);
    const bool hit = m <= (float)(Dp - r.tau);
    if (__builtin_expect(ballot(hit) != 0, 0)) {
      double nthr = thr;
      const double eo = uniform_f64(gp((const StepRec*)v.rec)[I.tab_off + t].eo);
      const double KE = thr - Dp * his + eo;
      replay<float>(v, b, I, t, p, valid, KE, nthr, lkey, lmask, pub, myc, lane);
      retune(nthr);
    }
  };
  auto flip_on = [&](double c) { Dp -= c; };
  auto flip_off = [&](double c) { Dp += c; };
  auto flip_sign = [&](bool off, double c) { Dp = __builtin_fma(off ? 1.0 : -1.0, c, Dp); };

  if (steps < 16) {
    HalfRow cur = row(0);
    for (uint32_t t = 0; t < steps; ++t) {
      if (t) {
        const int l = __builtin_ctz(t);
        flip_sign((t >> (l + 1)) & 1, myc[l * kWave + lane] * hs);
      }
      wait_rows();
      const HalfRow nxt = row(t + 1);
      __builtin_amdgcn_sched_barrier(0);
      body(t, cur);
      cur = nxt;
    }
    return;
  }
  // steps >= 16: unrolled by 8 as the float32 walk.  At the top of each step
  // the row of that step is waited for and the next row's loads are issued;
  // two rows are live (ev / od).  The cross field of the group's last flip
  // (bit 3 + CTZ(q + 1)) is read from LDS one step early, before a row load,
  // so the wait that covers it is the next step's row wait.
  HalfRow ev = row(0), od;
  wait_rows();
  od = row(1);
  __builtin_amdgcn_sched_barrier(0);
  body(0, ev);
  const uint32_t groups = steps >> 3;
  // steps 8q+1 .. 8q+6 of group q
  auto six = [&](uint32_t q) {
    const uint32_t t = 8 * q;
    wait_rows();
    ev = row(t + 2);
    __builtin_amdgcn_sched_barrier(0);
    flip_on(c0);
    body(t + 1, od);
    wait_rows();
    od = row(t + 3);
    __builtin_amdgcn_sched_barrier(0);
    flip_on(c1);
    body(t + 2, ev);
    wait_rows();
    ev = row(t + 4);
    __builtin_amdgcn_sched_barrier(0);
    flip_off(c0);
    body(t + 3, od);
    wait_rows();
    od = row(t + 5);
    __builtin_amdgcn_sched_barrier(0);
    flip_sign(q & 1, c2);
    body(t + 4, ev);
    wait_rows();
    ev = row(t + 6);
    __builtin_amdgcn_sched_barrier(0);
    flip_on(c0);
    body(t + 5, od);
    wait_rows();
    od = row(t + 7);
    __builtin_amdgcn_sched_barrier(0);
    flip_off(c1);
    body(t + 6, ev);
  };
  // every group but the last ends with steps 8q+7 and 8q+8 (the flip of bit
  // 3 + CTZ(q+1)); the last group, peeled, ends with step 8q+7
  if (paced) __builtin_amdgcn_s_setprio(3);
  for (uint32_t q = 0; q + 1 < groups; ++q) {
    six(q);
    const uint32_t t = 8 * q;
    wait_rows();
    const uint32_t t8 = t + 8;
    const int l8 = __builtin_ctz(t8);
    const double cl = myc[l8 * kWave + lane];
    __builtin_amdgcn_sched_barrier(0);
    ev = row(t8);
    __builtin_amdgcn_sched_barrier(0);
    flip_off(c0);
    body(t + 7, od);
    wait_rows();
    od = row(t8 + 1);
    __builtin_amdgcn_sched_barrier(0);
    flip_sign((t8 >> (l8 + 1)) & 1, cl * hs);
    body(t8, ev);
    if (((q + 1) & 7) == 0) {
      const double g = load_gthr(v, b);
      if (enc_key(g) < pub) pub = enc_key(g);
      if (g < thr) retune(g);
      if (paced) pace(q + 1, groups);
    }
  }
  six(groups - 1);
  wait_rows();
  flip_off(c0);
  body(8 * (groups - 1) + 7, od);
}

// ---- int32 walk with the int16 screen ---------------------------------------
//
// The same split and row layout (rows in 256-byte step slots) in exact int16
// arithmetic, for instances whose
// inner bound R_I is at most 32767 (then C', Tb, Ta and every partial sum of
// them are exact int16 values, and the screen decides exactly as the int32
// one).  Invalid lanes / inner states carry 32767 and saturating adds, so they
// can only cause a harmless replay.
typedef short s2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ s2 as_s2(uint32_t x) { return __builtin_bit_cast(s2, x); }

__device__ __forceinline__ int32_t int16_block_min(const HalfRow& r, const s2 (&C)[2][16]) {
  s2 m[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    s2 s[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const s2 x = as_s2(r.tb[c >> 1]);
      s[c] = __builtin_elementwise_add_sat(
          C[a][c], (c & 1) ? __builtin_shufflevector(x, x, 1, 1) : __builtin_shufflevector(x, x, 0, 0));
    }
#pragma unroll
    for (int w = 8; w > 0; w >>= 1)
#pragma unroll
      for (int c = 0; c < w; ++c) s[c] = __builtin_elementwise_min(s[c], s[c + w]);
    m[a] = __builtin_elementwise_add_sat(s[0], as_s2(r.ta[a]));
  }
  m[0] = __builtin_elementwise_min(m[0], m[1]);
  const s2 f = __builtin_elementwise_min(m[0], __builtin_shufflevector(m[0], m[0], 1, 0));
  return (int32_t)f.x;
}

__device__ __forceinline__ void walk_unit_i16(const Views& v, int b, const InstU& I, uint64_t local, double& lkey,
                                              uint64_t& lmask, uint64_t& pub, int64_t* myc, int lane,
                                              bool paced = false) {
  const bool valid = lane < (1 << I.L);
  const uint64_t p = (local << I.L) | (uint64_t)lane;
  // C'(j), j = c | a << 4, as int16 pairs (a, a + 2); invalid entries 32767
  const double g0 = load_gthr(v, b);  // issued first: its latency overlaps the set-up's
  s2 C16[2][16];
  const int64_t EP = lane_init_with<int32_t, 64, true>(v, b, I, local, valid, myc, lane, [&](int j, bool ok, int64_t cj) {
    C16[(j >> 4) & 1][j & 15][j >> 5] = (short)(ok ? cj : kInt16Limit);
  });

  if (enc_key(g0) < pub) pub = enc_key(g0);
  double thr = fmin(fmin(g0, I.big), readlane_f64(lkey, I.kp - 1));
  int32_t Dp = (int32_t)thr - (int32_t)EP;  // the int32 walk's Dp
  const uint32_t steps = 1u << I.no;
  const half_words_t rows = (half_words_t)((const HalfRow*)v.tab + I.tab_off * kInt16RowStride);
  const int32_t c0 = I.no > 0 ? (int32_t)myc[lane] : 0;
  const int32_t c1 = I.no > 1 ? (int32_t)myc[kWave + lane] : 0;
  const int32_t c2 = I.no > 2 ? (int32_t)myc[2 * kWave + lane] : 0;

  auto row = [&](uint32_t t) -> HalfRow {
    const half_words_t w = rows + (size_t)(t < steps ? t : steps - 1) * (kInt16RowStride * sizeof(HalfRow) / 4);
    HalfRow r;
#pragma unroll
    for (int c = 0; c < 8; ++c) r.tb[c] = w[c];
    r.ta[0] = w[8];
    r.ta[1] = w[9];
    r.neo = (int32_t)w[10];
    return r;
  };
  auto retune = [&](double nthr) {
    Dp += (int32_t)nthr - (int32_t)thr;
    thr = nthr;
  };
  auto body = [&](uint32_t t, const HalfRow& r) {
    const int32_t m = int16_block_min(r, C16);
    const bool hit = m <= Dp + r.neo;
    if (__builtin_expect(ballot(hit) != 0, 0)) {
      double nthr = thr;
      const int64_t KE = (int64_t)(int32_t)thr - (int64_t)Dp - (int64_t)r.neo;
      replay<int32_t>(v, b, I, t, p, valid, KE, nthr, lkey, lmask, pub, myc, lane);
      retune(nthr);
    }
  };
  auto flip_on = [&](int32_t c) { Dp -= c; };
  auto flip_off = [&](int32_t c) { Dp += c; };
  auto flip_sign = [&](bool off, int32_t c) { Dp += off ? c : -c; };

  if (steps < 16) {
    HalfRow cur = row(0);
    for (uint32_t t = 0; t < steps; ++t) {
      if (t) {
        const int l = __builtin_ctz(t);
        flip_sign((t >> (l + 1)) & 1, (int32_t)myc[l * kWave + lane]);
      }
      wait_rows();
      const HalfRow nxt = row(t + 1);
      __builtin_amdgcn_sched_barrier(0);
      body(t, cur);
      cur = nxt;
    }
    return;
  }
  // steps >= 16: the float32 walk's unrolled schedule (see walk_unit_h16)
  HalfRow ev = row(0), od;
  wait_rows();
  od = row(1);
  __builtin_amdgcn_sched_barrier(0);
  body(0, ev);
  const uint32_t groups = steps >> 3;
  auto six = [&](uint32_t q) {  // steps 8q+1 .. 8q+6
    const uint32_t t = 8 * q;
    wait_rows();
    ev = row(t + 2);
    __builtin_amdgcn_sched_barrier(0);
    flip_on(c0);
    body(t + 1, od);
    wait_rows();
    od = row(t + 3);
    __builtin_amdgcn_sched_barrier(0);
    flip_on(c1);
    body(t + 2, ev);
    wait_rows();
    ev = row(t + 4);
    __builtin_amdgcn_sched_barrier(0);
    flip_off(c0);
    body(t + 3, od);
    wait_rows();
    od = row(t + 5);
    __builtin_amdgcn_sched_barrier(0);
    flip_sign(q & 1, c2);
    body(t + 4, ev);
    wait_rows();
    ev = row(t + 6);
    __builtin_amdgcn_sched_barrier(0);
    flip_on(c0);
    body(t + 5, od);
    wait_rows();
    od = row(t + 7);
    __builtin_amdgcn_sched_barrier(0);
    flip_off(c1);
    body(t + 6, ev);
  };
  if (paced) __builtin_amdgcn_s_setprio(3);
  for (uint32_t q = 0; q + 1 < groups; ++q) {
    six(q);
    const uint32_t t = 8 * q;
    wait_rows();
    const uint32_t t8 = t + 8;
    const int l8 = __builtin_ctz(t8);
    const int32_t cl = (int32_t)myc[l8 * kWave + lane];
    __builtin_amdgcn_sched_barrier(0);
    ev = row(t8);
    __builtin_amdgcn_sched_barrier(0);
    flip_off(c0);
    body(t + 7, od);
    wait_rows();
    od = row(t8 + 1);
    __builtin_amdgcn_sched_barrier(0);
    flip_sign((t8 >> (l8 + 1)) & 1, cl);
    body(t8, ev);
    if (((q + 1) & 7) == 0) {
      const double g = load_gthr(v, b);
      if (enc_key(g) < pub) pub = enc_key(g);
      if (g < thr) retune(g);
      if (paced) pace(q + 1, groups);
    }
  }
  six(groups - 1);
  wait_rows();
  flip_off(c0);
  body(8 * (groups - 1) + 7, od);
}

template <class E, bool kHalf>
__device__ __forceinline__ void walk_topk_body(const Views& v) {
  using W = typename Ar<E>::W;
  __shared__ W ctab[kWavesPerBlock][kWaveRows * kWave];
  const int lane = threadIdx.x & 63;
  W* myc = ctab[threadIdx.x >> 6];
  const uint64_t total_units = uniform_u64(gp((const Header*)v.hdr)->total_units);
  double lkey = __builtin_inf();
  uint64_t lmask = ~0ull;
  uint64_t pub = ~0ull;
  int cur = -1;
  WorkIter it(v, total_units);
  // about one unit per wave: pace the waves of a SIMD (see pace)
  const bool paced = total_units <= (uint64_t)gridDim.x * kWavesPerBlock;
  uint64_t u;
  while (it.next(v, lane, u)) {
    const int b = v.batch == 1 ? 0 : find_unit(v, u);
    if (b != cur) {
      if (cur >= 0) flush(v, cur, lkey, lmask, lane);
      lkey = __builtin_inf();
      lmask = ~0ull;
      pub = ~0ull;
      cur = b;
    }
    const InstU I = load_inst(v, b);
    if (I.status == 0) {
      const uint64_t local = u - (uint64_t)I.unit_begin + (uint64_t)I.local_off;
      if constexpr (std::is_same_v<E, int32_t>) {
        // int32 Q beyond the int32 walk's range: float64 tables, half screen
        if (uniform_i32(gp((const Inst*)v.inst)[b].wide)) {
          // the unit reads and writes the LDS rows as float64: keep the
          // compiler from moving int64 accesses of other units across it
          __asm__ volatile("" ::: "memory");
          walk_unit_h16<kInt16RowStride>(v, b, I, local, lkey, lmask, pub, (double*)myc, lane);
          __asm__ volatile("" ::: "memory");
          continue;
        }
      }
      if constexpr (kHalf && std::is_same_v<E, float>) {
        walk_unit_h16(v, b, I, local, lkey, lmask, pub, myc, lane, paced);
      } else if constexpr (kHalf) {
        // int16 screen where the instance's inner bound allows it
        if (uniform_f64(gp((const Inst*)v.inst)[b].hscale) != 0.0)
          walk_unit_i16(v, b, I, local, lkey, lmask, pub, myc, lane, paced);
        else
          walk_unit<E>(v, b, I, local, lkey, lmask, pub, myc, lane);
      } else {
        walk_unit<E>(v, b, I, local, lkey, lmask, pub, myc, lane);
      }
    }
  }
  if (cur >= 0) flush(v, cur, lkey, lmask, lane);
}

// Three waves per SIMD for the float32 / int32 screens; two for the float64
// walk (its 32-entry table and broadcast temporaries take 2x the VGPRs).
template <class E>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) walk_topk_kernel(Views v) {
  walk_topk_body<E, false>(v);
}
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) walk_topk_f64_kernel(Views v) {
  walk_topk_body<double, false>(v);
}
// The half-screen walks keep their step loops within 128 VGPRs (the rows are
// in scalar registers, C' is 32 packed pairs), so they run 4 waves per SIMD:
// the extra wave hides the scalar row loads, unit set-up and the serial tail
// of each step's minimum tree (float16: n=40 1.5 % faster, the 4096-instance
// batch 6 %; int16: n=32 int32 10 %); the set-up and replay paths spill.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) walk_topk_h16_kernel(Views v) {
  walk_topk_body<float, true>(v);
}
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) walk_topk_i16_kernel(Views v) {
  walk_topk_body<int32_t, true>(v);
}

}  // namespace

namespace {
int occupancy_blocks(const void* kernel) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}
}  // namespace

int walk_topk_blocks_per_cu(int dt, int h16) {
  // one query per kernel, cached (the answer is fixed for the code object)
  static int cache[5] = {0, 0, 0, 0, 0};
  const int i = (dt == kDtI32 && h16) ? 0 : dt == kDtI32 ? 1 : h16 ? 2 : dt_wide(dt) ? 3 : 4;
  if (!cache[i]) {
    const void* k = i == 0   ? (const void*)walk_topk_i16_kernel
                    : i == 1 ? (const void*)walk_topk_kernel<int32_t>
                    : i == 2 ? (const void*)walk_topk_h16_kernel
                    : i == 3 ? (const void*)walk_topk_f64_kernel
                             : (const void*)walk_topk_kernel<float>;
    cache[i] = occupancy_blocks(k);
  }
  return cache[i];
}

hipError_t launch_walk_topk(const Views& v, int dt, int waves, hipStream_t s) {
  const int blocks = max(1, (waves + kWavesPerBlock - 1) / kWavesPerBlock);
  if (dt == kDtI32 && v.h16)
    hipLaunchKernelGGL(walk_topk_i16_kernel, dim3(blocks), dim3(kBlock), 0, s, v);
  else if (dt == kDtI32)
    hipLaunchKernelGGL(walk_topk_kernel<int32_t>, dim3(blocks), dim3(kBlock), 0, s, v);
  else if (v.h16)  // float32, float64 and int64 Q
    hipLaunchKernelGGL(walk_topk_h16_kernel, dim3(blocks), dim3(kBlock), 0, s, v);
  else if (dt_wide(dt))
    hipLaunchKernelGGL(walk_topk_f64_kernel, dim3(blocks), dim3(kBlock), 0, s, v);
  else
    hipLaunchKernelGGL(walk_topk_kernel<float>, dim3(blocks), dim3(kBlock), 0, s, v);
  return hipGetLastError();
}

}  // namespace qbf
