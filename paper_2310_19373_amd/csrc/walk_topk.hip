// Persistent top-k enumeration kernel (the hot path).
//
// Each wave pulls work units from a queue.  A unit fixes the tile bits; lane l
// fixes the lane bits (the prefix split of Sec. 3.1: 2^(L+tb) independent
// sub-walks whose results are min-combined).  Per lane and unit:
//
//   * lane init: E_P, the per-lane inner table C'(j) = E_I(j) + X_PI(p, j)
//     (64 entries, float32 or int32, in VGPRs) and the per-lane cross fields
//     c_l = sum_{v in prefix} S_{l v} x_v of the outer bits (LDS);
//   * outer walk over t = 0 .. 2^no - 1 in reflected Gray order: step t flips
//     bit l = CTZ(t) (Sec. 2.2), turning it on iff bit l+1 of t is 0; the
//     per-lane scalar KE = E_P + X_PO + E_O moves by +-c_l plus the uniform
//     E_O(g(t)) (Eq. 3 restricted to the prefix/outer cross terms);
//   * 64 inner states per step: e_j = C'(j) + T'(g(t); j), with T' broadcast
//     across each 16-lane row by DPP (one v_add_*_dpp per state) and folded by
//     v_min3 (half an instruction per state);
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
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"
#include "wave.hpp"

namespace qbf {

namespace {

template <class E>
struct Ar;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

template <>
struct Ar<float> {
  using W = double;
  using V = f32x4;
  __device__ static float inv() { return __builtin_inff(); }
  __device__ static float mn(float a, float b) { return __builtin_fminf(a, b); }
};
template <>
struct Ar<int32_t> {
  using W = int64_t;
  using V = i32x4;
  __device__ static int32_t inv() { return kIntInvalid; }
  __device__ static int32_t mn(int32_t a, int32_t b) { return a < b ? a : b; }
};

// acc = min(acc, C'(16K+Q) + T'(16K+Q)) over Q = 0..15 for register K of the
// row-replicated T' table.
template <int K, int Q, class E>
__device__ __forceinline__ void block_min(E& acc, E t, const E* C) {
  const E e0 = row_bcast<Q>(t) + C[16 * K + Q];
  const E e1 = row_bcast<Q + 1>(t) + C[16 * K + Q + 1];
  acc = Ar<E>::mn(Ar<E>::mn(acc, e0), e1);
  if constexpr (Q + 2 < 16) block_min<K, Q + 2>(acc, t, C);
}

__device__ __forceinline__ int find_unit(const Views& v, uint64_t u) {
  const gptr<const Inst> inst = gp((const Inst*)v.inst);
  int lo = 0, hi = v.batch;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((uint64_t)inst[mid].unit_begin <= u) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Instance fields as provably uniform (SGPR) values: the kernel's own atomics
// keep the compiler from proving the loads unclobbered, so force uniformity.
struct InstU {
  int n, B, L, no, kp, status;
  int64_t unit_begin, tab_off, slot_off, slot_cap;
  double big;
};

__device__ __forceinline__ InstU load_inst(const Views& v, int b) {
  const gptr<const Inst> I = gp((const Inst*)v.inst) + b;
  InstU r;
  r.n = uniform_i32(I->n);
  r.B = uniform_i32(I->B);
  r.L = uniform_i32(I->L);
  r.no = uniform_i32(I->no);
  r.kp = uniform_i32(I->kprime);
  r.status = uniform_i32(I->status);
  r.unit_begin = (int64_t)uniform_u64((uint64_t)I->unit_begin);
  r.tab_off = (int64_t)uniform_u64((uint64_t)I->tab_off);
  r.slot_off = (int64_t)uniform_u64((uint64_t)I->slot_off);
  r.slot_cap = (int64_t)uniform_u64((uint64_t)I->slot_cap);
  r.big = uniform_f64(I->big);
  return r;
}

__device__ __forceinline__ double load_gthr(const Views& v, int b) {
  const uint64_t g = __hip_atomic_load(gp(v.gthr) + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return dec_key(uniform_u64(g));
}

// Writes the wave's list to the next free slot of instance b.  A count above
// the slot capacity is reported by the finalize kernel (it cannot happen: a
// wave flushes an instance at most once per contiguous run of its units).
__device__ void flush(const Views& v, int b, double lkey, uint64_t lmask, int lane) {
  const InstU I = load_inst(v, b);
  uint32_t slot = 0;
  if (lane == 0) slot = atomicAdd(v.flushcnt + b, 1u);
  slot = readlane_u32(slot, 0);
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
                                       uint64_t& pub, int lane) {
  using W = typename Ar<E>::W;
  const int pos0 = I.B + I.no;
  const int64_t nm = v.nmax;
  const gptr<const W> qs = gp((const W*)v.qs) + (int64_t)b * nm * nm;
  const gptr<const W> ei = gp((const W*)v.ei) + (int64_t)b * 64;
  W cI[6] = {0, 0, 0, 0, 0, 0};
  for (int a = pos0; a < I.n; ++a) {
    if (!((p >> (a - pos0)) & 1)) continue;
#pragma unroll
    for (int u = 0; u < 6; ++u)
      if (u < I.B) cI[u] += qs[(int64_t)u * nm + a];
  }
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
  const int pos0 = I.B + I.no;
  const bool valid = lane < (1 << I.L);
  const uint64_t p = (local << I.L) | (uint64_t)lane;
  const int64_t nm = v.nmax;
  const gptr<const W> qs = gp((const W*)v.qs) + (int64_t)b * nm * nm;
  const gptr<const W> ei = gp((const W*)v.ei) + (int64_t)b * 64;

  // ---- lane init: prefix energy, inner cross fields, outer cross fields
  W EP = 0;
  W cI[6] = {0, 0, 0, 0, 0, 0};
  for (int a = pos0; a < I.n; ++a) {
    if (!((p >> (a - pos0)) & 1)) continue;
    W row = qs[(int64_t)a * nm + a];
    for (int c = a + 1; c < I.n; ++c)
      if ((p >> (c - pos0)) & 1) row += qs[(int64_t)a * nm + c];
    EP += row;
#pragma unroll
    for (int u = 0; u < 6; ++u)
      if (u < I.B) cI[u] += qs[(int64_t)u * nm + a];
  }
  for (int l = 0; l < I.no; ++l) {
    W c = 0;
    for (int a = pos0; a < I.n; ++a)
      if ((p >> (a - pos0)) & 1) c += qs[(int64_t)(I.B + l) * nm + a];
    myc[l * kWave + lane] = c;
  }
  E C[kInnerStates];
#pragma unroll
  for (int j = 0; j < kInnerStates; ++j) {
    W cj = ei[j];
#pragma unroll
    for (int u = 0; u < 6; ++u)
      if ((j >> u) & 1) cj += cI[u];
    C[j] = (valid && j < (1 << I.B)) ? (E)cj : Ar<E>::inv();
  }

  double thr = fmin(fmin(load_gthr(v, b), I.big), readlane_f64(lkey, I.kp - 1));
  const uint32_t steps = 1u << I.no;
  const int q = lane & 15;
  const gptr<const V> trow = (gptr<const V>)(gp((const E*)v.tab) + I.tab_off * kInnerStates) + q;
  const gptr<const StepRec> rec = gp((const StepRec*)v.rec) + I.tab_off;
  // Operands of step t, loaded one step ahead: T' row, E_O (or -E_O), and the
  // cross field c_l of the bit flipped into step t.  Indices are clamped so the
  // loads are unconditional (the clamped values are never used).
  struct Ops {
    V tv;
    double eo;
    int32_t neo;
    W c;
  };
  auto load = [&](uint32_t t) {
    const uint32_t tt = t < steps ? t : steps - 1;
    Ops o;
    o.tv = trow[tt * 16];
    if constexpr (std::is_same_v<E, float>) o.eo = rec[tt].eo;
    else o.neo = rec[tt].neo;
    o.c = myc[(tt ? __builtin_ctz(tt) : 0) * kWave + lane];
    return o;
  };

  if constexpr (std::is_same_v<E, float>) {
    double K = EP;  // E_P + X_PO(p, g(t))
    // One outer step: flip, block minimum over the 64 inner states, filter.
    auto step = [&](uint32_t t, const Ops& o) {
      if (t != 0) {
        const double sg = ((t >> (__builtin_ctz(t) + 1)) & 1) ? -1.0 : 1.0;
        K = __builtin_fma(sg, o.c, K);
      }
      const double KE = K + o.eo;
      const double D = thr - KE;
      float acc = __builtin_inff();
      block_min<0, 0>(acc, o.tv.x, C);
      block_min<1, 0>(acc, o.tv.y, C);
      block_min<2, 0>(acc, o.tv.z, C);
      block_min<3, 0>(acc, o.tv.w, C);
      if (__builtin_expect(ballot((double)acc <= D) != 0, 0))
        replay<E>(v, b, I, t, p, valid, KE, thr, lkey, lmask, pub, lane);
      if ((t & 63) == 63) thr = fmin(thr, load_gthr(v, b));
    };
    Ops oa = load(0);
    for (uint32_t t = 0; t < steps; t += 2) {
      // steps is 1 or even; the two operand buffers alternate
      const Ops ob = load(t + 1);
      step(t, oa);
      if (t + 1 >= steps) break;
      oa = load(t + 2);
      step(t + 1, ob);
    }
  } else {
    int32_t NK = -(int32_t)EP;  // -(E_P + X_PO(p, g(t)))
    int32_t thr_i = (int32_t)thr;
    auto step = [&](uint32_t t, const Ops& o) {
      if (t != 0) {
        const int32_t c = (int32_t)o.c;
        NK = ((t >> (__builtin_ctz(t) + 1)) & 1) ? NK + c : NK - c;
      }
      const int32_t D = thr_i + NK + o.neo;
      int32_t acc = kIntInvalid;
      block_min<0, 0>(acc, o.tv.x, C);
      block_min<1, 0>(acc, o.tv.y, C);
      block_min<2, 0>(acc, o.tv.z, C);
      block_min<3, 0>(acc, o.tv.w, C);
      if (__builtin_expect(ballot(acc <= D) != 0, 0)) {
        replay<E>(v, b, I, t, p, valid, -(int64_t)NK - (int64_t)o.neo, thr, lkey, lmask, pub, lane);
        thr_i = (int32_t)thr;
      }
      if ((t & 63) == 63) {
        thr = fmin(thr, load_gthr(v, b));
        thr_i = (int32_t)thr;
      }
    };
    Ops oa = load(0);
    for (uint32_t t = 0; t < steps; t += 2) {
      const Ops ob = load(t + 1);
      step(t, oa);
      if (t + 1 >= steps) break;
      oa = load(t + 2);
      step(t + 1, ob);
    }
  }
}

template <class E>
__global__ void __launch_bounds__(kBlock) walk_topk_kernel(Views v) {
  using W = typename Ar<E>::W;
  __shared__ W ctab[kWavesPerBlock][kMaxOuter * kWave];
  const int lane = threadIdx.x & 63;
  W* myc = ctab[threadIdx.x >> 6];
  const uint64_t total_units = uniform_u64(gp((const Header*)v.hdr)->total_units);
  double lkey = __builtin_inf();
  uint64_t lmask = ~0ull;
  uint64_t pub = ~0ull;
  int cur = -1;
  for (;;) {
    uint64_t u = 0;
    if (lane == 0) u = atomicAdd((unsigned long long*)&v.hdr->unit_counter, 1ull);
    u = readlane_u64(u, 0);
    if (u >= total_units) break;
    const int b = v.batch == 1 ? 0 : find_unit(v, u);
    if (b != cur) {
      if (cur >= 0) flush(v, cur, lkey, lmask, lane);
      lkey = __builtin_inf();
      lmask = ~0ull;
      pub = ~0ull;
      cur = b;
    }
    const InstU I = load_inst(v, b);
    if (I.status == 0) walk_unit<E>(v, b, I, u - (uint64_t)I.unit_begin, lkey, lmask, pub, myc, lane);
  }
  if (cur >= 0) flush(v, cur, lkey, lmask, lane);
}

}  // namespace

hipError_t launch_walk_topk(const Views& v, bool is_int, int waves, hipStream_t s) {
  const int blocks = max(1, (waves + kWavesPerBlock - 1) / kWavesPerBlock);
  if (is_int)
    hipLaunchKernelGGL(walk_topk_kernel<int32_t>, dim3(blocks), dim3(kBlock), 0, s, v);
  else
    hipLaunchKernelGGL(walk_topk_kernel<float>, dim3(blocks), dim3(kBlock), 0, s, v);
  return hipGetLastError();
}

}  // namespace qbf
