// Shared pieces of the enumeration kernels: arithmetic traits, uniform
// instance fields, the per-lane init of the block-table walk and the
// DPP-broadcast block minimum.
#pragma once
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"
#include "wave.hpp"

namespace qbf {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <class E>
struct Ar;
// W: exact accumulation type; V: one lane's 16-byte share of a 256-byte T'
// row; NB: inner states per lane (the row holds NB entries of E).
template <>
struct Ar<float> {
  using W = double;
  using V = f32x4;
  static constexpr int NB = 64;
  __device__ static float inv() { return __builtin_inff(); }
  __device__ static float mn(float a, float b) { return __builtin_fminf(a, b); }
};
template <>
struct Ar<int32_t> {
  using W = int64_t;
  using V = i32x4;
  static constexpr int NB = 64;
  __device__ static int32_t inv() { return kIntInvalid; }
  __device__ static int32_t mn(int32_t a, int32_t b) { return a < b ? a : b; }
};
template <>
struct Ar<double> {
  using W = double;
  using V = f64x2;
  static constexpr int NB = 32;
  __device__ static double inv() { return __builtin_inf(); }
  __device__ static double mn(double a, double b) { return __builtin_fmin(a, b); }
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

// float64 walk: acc = min(acc, C'(16K+Q) + T'(16K+Q)) over Q = 0..15.  The
// sixteen row broadcasts are 64-bit DPP moves (gfx950 has no DPP form of
// v_add_f64), one asm block so that one s_nop covers the hazard of a VALU
// write to t just before; then one v_add_f64 and one v_min_f64 per state.
template <int K>
__device__ __forceinline__ void block_min_f64(double& acc, double t, const double* C) {
  double b[16];
  asm("s_nop 1\n"
      "v_mov_b64_dpp %0, %16 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %1, %16 row_newbcast:1 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %2, %16 row_newbcast:2 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %3, %16 row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %4, %16 row_newbcast:4 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %5, %16 row_newbcast:5 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %6, %16 row_newbcast:6 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %7, %16 row_newbcast:7 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %8, %16 row_newbcast:8 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %9, %16 row_newbcast:9 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %10, %16 row_newbcast:10 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %11, %16 row_newbcast:11 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %12, %16 row_newbcast:12 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %13, %16 row_newbcast:13 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %14, %16 row_newbcast:14 row_mask:0xf bank_mask:0xf\n"
      "v_mov_b64_dpp %15, %16 row_newbcast:15 row_mask:0xf bank_mask:0xf"
      : "=&v"(b[0]), "=&v"(b[1]), "=&v"(b[2]), "=&v"(b[3]), "=&v"(b[4]), "=&v"(b[5]), "=&v"(b[6]),
        "=&v"(b[7]), "=&v"(b[8]), "=&v"(b[9]), "=&v"(b[10]), "=&v"(b[11]), "=&v"(b[12]), "=&v"(b[13]),
        "=&v"(b[14]), "=&v"(b[15])
      : "v"(t));
#pragma unroll
  for (int q = 0; q < 16; q += 2)
    acc = __builtin_fmin(__builtin_fmin(acc, b[q] + C[16 * K + q]), b[q + 1] + C[16 * K + q + 1]);
}

__device__ __forceinline__ int find_unit(const Views& v, uint64_t u) {
  if (v.umap) return uniform_i32((int)gp((const uint32_t*)v.umap)[u]);
  const gptr<const Inst> inst = gp((const Inst*)v.inst);
  int lo = 0, hi = v.batch;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((uint64_t)inst[mid].unit_begin <= u) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Takes `want` units from queue segment `sg` and returns the first, identical
// in all lanes.  Every lane issues the atomic (increment `want` from lane 0, 0
// from the others) and the result of the first lane is broadcast: there is no
// lane-divergent branch around the pull, so the loop exit it controls is
// uniform.  Must be called with all lanes active and a uniform `want`.
__device__ __forceinline__ uint64_t take_units(const Views& v, int sg, int lane, uint64_t want) {
  const uint64_t r = atomicAdd((unsigned long long*)&v.hdr->seg[sg].next, lane == 0 ? want : 0ull);
  return uniform_u64(r);
}

// Work distribution of the persistent walks, in runs of consecutive units.
// Dynamic (v.dyn): the unit range is cut into kXcds segments, and a wave works
// on the segment of its XCD (workgroup index mod kXcds) first.
//   * Its first run is assigned statically: the planner started each
//     segment's counter past one run of `cap` units per wave of that segment
//     (the waves of workgroups x, x + 8, ... in order), so the grid starts
//     without a burst of atomics on eight counters.
//   * Later runs are pulled with an atomic add (guided self-scheduling: a pull
//     takes min(cap, rest / (2 x waves per segment)) units, at least 1, rest
//     being what the segment had left after the wave's previous pull, so runs
//     shrink towards the end).
//   * Near a segment's end, and after a pull that found it empty, the wave
//     first reads the eight counters with one lane-parallel load and pulls
//     from the first later segment that still has units, or stops: a drained
//     segment is not hit by one atomic from every wave of the grid.
// A wave only moves on to later segments, so its units increase
// monotonically.  Static (!v.dyn): wave w of G takes runs w, w+G, ... of cap
// units.  Either way a wave meets each instance in one contiguous stretch,
// and its candidate list carries over between the units of a run.
//
// The static first runs assume the grid the planner was told (Header.waves
// waves, in blocks of kWavesPerBlock): every launch of a walk uses that grid.
struct WorkIter {
  uint64_t total, cap, want, waves2, u = 0, u_end = 0, next_static, seg_end, left;
  int64_t stride;
  int sg;
  bool dyn, first;
  __device__ WorkIter(const Views& v, uint64_t total_units) {
    const gptr<const Header> h = gp((const Header*)v.hdr);
    total = total_units;
    cap = (uint64_t)(uint32_t)uniform_i32(h->chunk);
    want = cap;
    dyn = v.dyn != 0;
    first = true;
    next_static = (uint64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    stride = (int64_t)gridDim.x * kWavesPerBlock;
    const uint64_t per_seg = (uint64_t)stride / kXcds;
    waves2 = 2 * (per_seg > 0 ? per_seg : 1);
    sg = (int)(blockIdx.x % kXcds);
    seg_end = uniform_u64(h->seg[sg].end);
    left = ~0ull;
  }
  // The first run of this wave: units [begin + rank * cap, + cap) of its
  // segment, clipped to the segment (empty for a wave beyond the planned
  // grid or a segment with fewer units than waves).
  __device__ __forceinline__ bool static_run(const Views& v) {
    const uint64_t pw = (uint64_t)(uint32_t)uniform_i32(gp((const Header*)v.hdr)->waves);
    const uint64_t blocks = pw / kWavesPerBlock;
    const uint64_t bi = blockIdx.x;
    if (bi >= blocks) return false;
    const uint64_t x = (uint64_t)sg;
    const uint64_t rank = (bi / kXcds) * kWavesPerBlock + (threadIdx.x >> 6);
    const uint64_t b0 = total * x / kXcds;
    // units the segment keeps for pulls after the static runs (as the planner)
    const uint64_t wx = blocks > x ? (blocks - x + kXcds - 1) / kXcds * kWavesPerBlock : 0;
    const uint64_t sdone = b0 + wx * cap < seg_end ? b0 + wx * cap : seg_end;
    left = seg_end - sdone;
    const uint64_t c = b0 + rank * cap;
    if (c >= seg_end) return false;
    u = c;
    u_end = c + cap < seg_end ? c + cap : seg_end;
    return true;
  }
  __device__ __forceinline__ bool next(const Views& v, int lane, uint64_t& unit) {
    if (u >= u_end) {
      if (dyn) {
        if (first) {
          first = false;
          if (static_run(v)) {
            unit = u++;
            return true;
          }
        }
        for (;;) {  // every value here is wave-uniform
          if (uniform_u64(left) <= uniform_u64(waves2) * cap) {
            // near or past the end of the segment: look at all counters
            const gptr<QueueSeg> seg = gp(v.hdr->seg);
            uint64_t nx = ~0ull, ex = 0;
            if (lane < kXcds) {
              nx = __hip_atomic_load(&seg[lane].next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              ex = seg[lane].end;
            }
            const uint64_t avail = ballot(lane < kXcds && lane >= uniform_i32(sg) && nx < ex);
            if (!avail) return false;
            const int s = __builtin_ctzll(avail);
            if (s != uniform_i32(sg)) {
              sg = s;
              seg_end = readlane_u64(ex, s);
              want = cap;
            }
            left = ~0ull;
          }
          const int s = uniform_i32(sg);
          const uint64_t w = uniform_u64(want);
          const uint64_t e = uniform_u64(seg_end);
          const uint64_t c = take_units(v, s, lane, w);
          if (c < e) {
            u = c;
            u_end = c + w < e ? c + w : e;
            left = e - u_end;
            const uint64_t share = left / waves2;
            want = share < 1 ? 1 : (share > cap ? cap : share);
            break;
          }
          left = 0;  // drained: the next round looks before it pulls
        }
      } else {
        const uint64_t c = next_static;
        next_static += (uint64_t)stride;
        u = c * cap;
        if (u >= total) return false;
        u_end = u + cap < total ? u + cap : total;
      }
    }
    unit = u++;
    return true;
  }
};

// Instance fields as provably uniform (SGPR) values: the kernel's own atomics
// keep the compiler from proving the loads unclobbered, so force uniformity.
struct InstU {
  int n, B, L, no, kp, status;
  int64_t unit_begin, local_off, tab_off, slot_off, slot_cap;
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
  r.local_off = (int64_t)uniform_u64((uint64_t)I->local_off);
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

// Per-lane init of a work unit.  The lane owns the prefix p: its lane bits
// (positions B+no ..) and the unit's tile bits (positions B+no+L ..).  Fills
//   C'(j) = E_I(j) + X_PI(p, j)  for the 64 (NB) inner states (invalid lanes and
//           inner states get the type's sentinel),
//   LDS rows 0..no-1:   c_l = sum_{v in prefix} S_{B+l, v} x_v  (outer cross fields),
//   LDS rows kCIRow+u:  cI_u = sum_{v in prefix} S_{u, v} x_v   (inner cross fields),
// and returns E_P(p).  The lane-bit parts come from the instance's lane table;
// the tile-bit parts are summed lane-parallel (lane t takes row t, lane t also
// tile row t for E_tile) with independent loads, and exchanged through LDS.
//
// lane_init_with hands each inner entry to sink(j, ok, C'(j)) (ok: a valid
// lane and inner state) instead of storing a table, so a caller can keep the
// entries in another form without the 64-entry table ever being live.
template <class E, int NB, bool kLaneEI = false, class Sink>
__device__ __forceinline__ typename Ar<E>::W lane_init_with(const Views& v, int b, const InstU& I, uint64_t local,
                                                            bool valid, typename Ar<E>::W* myc, int lane,
                                                            Sink&& sink) {
  using W = typename Ar<E>::W;
  const int pos0 = I.B + I.no;
  const int tp0 = pos0 + I.L;  // first tile bit
  const int tb = I.n - tp0;
  const int64_t nm = v.nmax;
  const gptr<const W> qs = gp((const W*)v.qs) + (int64_t)b * nm * nm;
  const gptr<const W> ei = gp((const W*)v.ei) + (int64_t)b * 64;
  // kLaneEI (the half-width screens, whose set-up has registers to spare
  // before C' exists): the lane record's energy and inner cross fields and
  // this lane's E_I entry are read first, unconditionally (the record's
  // unused fields are zero), so that their latency overlaps the tile rows'
  // instead of following it one load at a time: [0] lane-bit energy, [1 + u]
  // inner cross field u.  The other walks read them where they are used (their
  // step loops hold 64-entry tables, and longer-lived set-up values spill).
  const gptr<const W> lt = gp((const W*)v.lt) + ((int64_t)b * 64 + lane) * kLaneRec;
  W lrec[7];
  if constexpr (kLaneEI) {
#pragma unroll
    for (int i = 0; i < 7; ++i) lrec[i] = lt[i];
  }
  const W eil = (kLaneEI && lane < NB) ? ei[lane] : (W)0;
  // tile sums: S (lane t < tp0) = sum_{set tile bits k} S(t, tp0+k);
  // R (tile row t = lane, bit t set) = sum_{set tile bits k >= t} Q(tp0+t, tp0+k)
  W S = 0, R = 0;
  const bool xt = lane < tb && ((local >> lane) & 1);
  const int64_t srow = (int64_t)(lane < tp0 ? lane : 0) * nm;
  const int64_t rrow = (int64_t)(tp0 + (lane < tb ? lane : 0)) * nm;
  for (int k0 = 0; k0 < tb; k0 += 8) {
    W s8[8], r8[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) {  // independent loads, clamped addresses
      const int kc = k0 + d < tb ? k0 + d : tb - 1;
      s8[d] = qs[srow + tp0 + kc];
      r8[d] = qs[rrow + tp0 + kc];
    }
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const int k = k0 + d;
      const bool xk = k < tb && ((local >> k) & 1);
      if (xk && lane < tp0) S += s8[d];
      if (xk && xt && lane <= k) R += r8[d];
    }
  }
  W etile = R;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) etile += __shfl_xor(etile, o);
  if constexpr (std::is_same_v<W, double>) etile = uniform_f64(etile);
  else etile = (W)uniform_u64((uint64_t)etile);
  myc[kTileRow * kWave + lane] = S;
  // lane record + tile sums
  if constexpr (!kLaneEI) {
    lrec[0] = lt[0];
#pragma unroll
    for (int u = 0; u < 6; ++u) lrec[1 + u] = u < I.B ? lt[1 + u] : (W)0;
  }
  W EP = etile + lrec[0];
  for (int a = 0; a < I.L; ++a)
    if ((lane >> a) & 1) EP += myc[kTileRow * kWave + pos0 + a];
  W cI[6];
#pragma unroll
  for (int u = 0; u < 6; ++u) {
    cI[u] = u < I.B ? lrec[1 + u] + myc[kTileRow * kWave + u] : (W)0;
    myc[(kCIRow + u) * kWave + lane] = cI[u];
  }
  if constexpr (kLaneEI) {  // outer cross fields: all loads in flight together, then the stores
    W lo[kMaxOuter];
#pragma unroll
    for (int l = 0; l < kMaxOuter; ++l) lo[l] = lt[8 + l];
#pragma unroll
    for (int l = 0; l < kMaxOuter; ++l)
      if (l < I.no) myc[l * kWave + lane] = lo[l] + myc[kTileRow * kWave + I.B + l];
  } else {
    for (int l = 0; l < I.no; ++l) myc[l * kWave + lane] = lt[8 + l] + myc[kTileRow * kWave + I.B + l];
  }
  // kLaneEI: lane j loaded E_I(j) above (one coalesced load) and the loop
  // reads it back by lane, for kernels at 128 VGPRs where 64 entries loaded
  // per lane (128 VGPRs in flight) would spill
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    W cj;
    if constexpr (!kLaneEI) cj = ei[j];
    else if constexpr (std::is_same_v<W, double>) cj = readlane_f64(eil, j);
    else cj = readlane_i64(eil, j);
#pragma unroll
    for (int u = 0; u < 6; ++u)
      if ((j >> u) & 1) cj += cI[u];
    sink(j, valid && j < (1 << I.B), cj);
  }
  return EP;
}

template <class E, int NB>
__device__ __forceinline__ typename Ar<E>::W lane_init(const Views& v, int b, const InstU& I, uint64_t local,
                                                       bool valid, typename Ar<E>::W* myc, int lane, E (&C)[NB]) {
  using W = typename Ar<E>::W;
  return lane_init_with<E, NB>(v, b, I, local, valid, myc, lane,
                               [&](int j, bool ok, W cj) { C[j] = ok ? (E)cj : Ar<E>::inv(); });
}

}  // namespace qbf
