// Planner and table builders.
//
// plan_kernel    : bit split of every instance, work-unit / table / slot offsets,
//                  queue and threshold reset (written by a kernel, so that a
//                  captured graph replays it without memset nodes).
// prep_inst      : work unit -> instance map, symmetric copy of Q (the qua/lin split of Sec. 3: off-diagonal
//                  S = triu(Q,1) + triu(Q,1)^T, diagonal d = diag(Q)), sum |Q|,
//                  validation, and the inner-bit energies E_I(j).
// prep_walk      : one launch of three independent roles per instance: the
//                  threshold seed (greedy descents), the lane table, and per
//                  outer Gray step t the uniform table T'(g(t); j) with the
//                  scalars E_O(g(t)), H_u(g(t)).
#include <math.h>

#include <type_traits>

#include "common.hpp"
#include "dpp.hpp"
#include "launch.hpp"
#include "wave.hpp"

namespace qbf {

namespace {

struct Split {
  int B, L, no, tb;
  int64_t units, steps;
};

__device__ Split split_bits(int n, const PlanParams& pp) {
  Split s;
  s.B = min(pp.inner, n);
  s.L = min(pp.lane_bits, n - s.B);
  const int rest = n - s.B - s.L;
  s.no = max(0, min(pp.no_max, rest - max(pp.ub_min, pp.range_bits)));
  s.tb = rest - s.no;
  s.units = int64_t(1) << s.tb;
  s.steps = int64_t(1) << s.no;
  if (pp.range_bits > 0) {  // the prefix range as a contiguous range of units
    const int shift = s.tb - pp.range_bits;
    s.units = shift >= 0 ? (pp.range_end - pp.range_begin) << shift : 0;
  }
  return s;
}

__global__ void __launch_bounds__(1024) plan_kernel(Views v, const int32_t* ns, int n_single, const float* beta,
                                                    PlanParams pp) {
  __shared__ int64_t su[1024], ss[1024], sl[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int batch = v.batch;
  const int per = (batch + nt - 1) / nt;
  const int b0 = min(batch, tid * per), b1 = min(batch, b0 + per);
  int64_t lu = 0, ls = 0, lsl = 0;
  for (int b = b0; b < b1; ++b) {
    const int n = ns ? ns[b] : n_single;
    if (n < 1 || n > v.nmax || n > 63) continue;
    const Split s = split_bits(n, pp);
    lu += s.units;
    ls += s.steps;
    lsl += min<int64_t>(s.units, pp.waves);
  }
  su[tid] = lu;
  ss[tid] = ls;
  sl[tid] = lsl;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {
    int64_t a = 0, c = 0, d = 0;
    if (tid >= off) {
      a = su[tid - off];
      c = ss[tid - off];
      d = sl[tid - off];
    }
    __syncthreads();
    su[tid] += a;
    ss[tid] += c;
    sl[tid] += d;
    __syncthreads();
  }
  int64_t cu = su[tid] - lu, cs = ss[tid] - ls, csl = sl[tid] - lsl;
  for (int b = b0; b < b1; ++b) {
    const int n = ns ? ns[b] : n_single;
    Inst I = {};
    I.n = n;
    I.kprime = pp.kprime;
    I.sign = (beta && beta[b] < 0.0f) ? -1.0 : 1.0;
    if (n < 1 || n > v.nmax || n > 63) {
      I.status = kErrArg;
      I.unit_begin = cu;
      I.tab_off = cs;
      I.slot_off = csl;
    } else {
      const Split s = split_bits(n, pp);
      I.B = s.B;
      I.L = s.L;
      I.no = s.no;
      I.tb = s.tb;
      I.units = s.units;
      I.unit_begin = cu;
      I.local_off = pp.range_bits > 0 ? pp.range_begin << (s.tb - pp.range_bits) : 0;
      if (beta && !isfinite(beta[b])) I.status = kErrNonfinite;  // the walks skip the instance
      I.seed_fix = pp.range_bits > 0 ? pp.range_bits : 0;
      if (pp.range_bits > s.tb) I.status = kErrArg;  // the host checks this; kept as a guard
      I.tab_off = cs;
      I.slot_off = csl;
      I.slot_cap = min<int64_t>(s.units, pp.waves);
      cu += s.units;
      cs += s.steps;
      csl += I.slot_cap;
    }
    v.inst[b] = I;
    v.gthr[b] = enc_key(__builtin_inf());
    v.flushcnt[b] = 0;
  }
  if (tid == nt - 1) {
    const uint64_t tu = (uint64_t)su[nt - 1];
    // about four pulls per wave or more, so the queue balances the tail
    int64_t c = su[nt - 1] / ((int64_t)(pp.waves > 0 ? pp.waves : 1) * 4);
    if (c > pp.chunk_cap) c = pp.chunk_cap;
    if (c < 1) c = 1;
    v.hdr->chunk = (int32_t)c;
    // Each segment's counter starts past the static first runs of its waves
    // (one run of c units per wave of the workgroups x, x + 8, ...; see
    // WorkIter): the walk takes those without an atomic.
    const int64_t blocks = pp.waves / kWavesPerBlock;
    for (int x = 0; x < kXcds; ++x) {
      const uint64_t b0 = tu * (uint64_t)x / kXcds, b1 = tu * (uint64_t)(x + 1) / kXcds;
      const uint64_t wx = blocks > x ? (uint64_t)((blocks - x + kXcds - 1) / kXcds) * kWavesPerBlock : 0;
      const uint64_t first = b0 + wx * (uint64_t)c;
      v.hdr->seg[x].next = v.dyn ? (first < b1 ? first : b1) : b0;
      v.hdr->seg[x].end = b1;
    }
    v.hdr->total_units = tu;
    v.hdr->direct_count = 0;
    v.hdr->total_steps = ss[nt - 1];
    v.hdr->total_slots = sl[nt - 1];
    v.hdr->batch = batch;
    v.hdr->nmax = v.nmax;
    v.hdr->waves = pp.waves;
  }
}

template <class T>
__device__ double absd(T x) {
  return fabs((double)x);
}

// Scale and margin of the half-precision screen.  Every screened value and
// partial sum (C', Tb, Ta, C' + Tb, C' + Tb + Ta) is a partial sum of the inner
// rows, so at most R_I in magnitude; scaled by hs = 2^s with R_I hs in
// [2^12, 2^13) it stays far inside float16 range.  Five float16 roundings
// (relative 2^-11 each) and the float32 ones put the screened value within
// 5.01 * 2^-11 * R_I hs of hs times the float32 walk's; the threshold's
// float64 / float32 roundings add at most 2^-22 R_I hs + 2^-52 sum|Q| hs;
// float16 subnormals (or their flush) at most 5 * 2^-14.  hmargin covers all
// of it, so every block the float32 screen would pass also passes the half
// screen, and the float32 walk's error bound eps still holds.  (For the
// float64 walk the same bound holds against its float64 screen, so its eps
// and certificate are unchanged as well.)
__device__ void set_half_screen(Inst* I, double rI, double sa) {
  I->hscale = 1.0;
  if (rI > 0.0 && isfinite(rI)) {
    int e;
    frexp(rI, &e);  // R_I in [2^(e-1), 2^e)
    I->hscale = ldexp(1.0, 13 - e);
  }
  I->hmargin = I->hscale * (0x1p-8 * rI + 0x1p-50 * sa) + 0x1p-10;
}

// Qin: input element type; W: exact accumulation type of the tables; E: the
// walk's element type (float32 / int32 / float64), which sets the error bound.
template <class Qin, class W, class E>
__global__ void __launch_bounds__(256) prep_inst_kernel(Views v, const Qin* q, int64_t ldq, int64_t stride,
                                                        int inner) {
  __shared__ double red_a[256], red_r[256];
  __shared__ int red_bad[256], red_frac[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  Inst* I = &v.inst[b];
  // work unit -> instance map (for every instance with units, whatever its
  // status: the walks look the instance up before they check it)
  if (v.umap) {
    const int64_t ub = I->unit_begin, nu = I->units;
    for (int64_t u = tid; u < nu; u += blockDim.x)
      if (ub + u < v.umap_cap) v.umap[ub + u] = (uint32_t)b;
  }
  if (I->status != 0) return;
  const int n = I->n, nmax = v.nmax, B = I->B;
  const Qin* Q = q + (int64_t)b * stride;
  const double sgn = I->sign;
  double sabs = 0.0, rI = 0.0;
  int bad = 0, frac = 0;
  for (int idx = tid; idx < n * n; idx += blockDim.x) {  // sums and validation over i <= j
    const int i = idx / n, j = idx % n;
    if (j < i) continue;
    const Qin val = Q[(int64_t)i * ldq + j];
    if constexpr (std::is_floating_point_v<Qin>) {
      if (!isfinite(val)) bad = 1;
      if ((double)val != trunc((double)val)) frac = 1;
    }
    sabs += absd(val);
    if (i < B) rI += absd(val);
  }
  red_a[tid] = sabs;
  red_r[tid] = rI;
  red_bad[tid] = bad;
  red_frac[tid] = frac;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (tid < off) {
      red_a[tid] += red_a[tid + off];
      red_r[tid] += red_r[tid + off];
      red_bad[tid] |= red_bad[tid + off];
      red_frac[tid] |= red_frac[tid + off];
    }
    __syncthreads();
  }
  // int32 Q beyond the int32 walk's exact range (sum |Q| > 2^28) takes
  // float64 tables and the half-screen walk, exact for integer data with sum
  // |Q| <= 2^50 -- which every int32 Q satisfies (at most 2016 entries of
  // magnitude <= 2^31 for n <= 63)
  bool wide = false;
  if constexpr (std::is_same_v<E, int32_t>) wide = red_a[0] > (double)kIntSumLimit;
  // the symmetric copy (S off the diagonal, d on it), sign applied
  W* qs = (W*)v.qs + (int64_t)b * nmax * nmax;
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx % n;
    const Qin val = (i <= j) ? Q[(int64_t)i * ldq + j] : Q[(int64_t)j * ldq + i];
    if (wide) ((double*)qs)[(int64_t)i * nmax + j] = sgn * (double)val;
    else qs[(int64_t)i * nmax + j] = (W)(sgn * (double)val);
  }
  // E_I(j) for the inner bits, straight from Eq. 1 restricted to bits < B;
  // the inner block of Q (at most 6 x 6) is read once into LDS, one load per
  // thread, and the sums keep their order
  __shared__ W qin[6][6];
  if (tid < 36) {
    const int u = tid / 6, w = tid % 6;
    qin[u][w] = (u < B && w < B && u <= w) ? (W)(sgn * (double)Q[(int64_t)u * ldq + w]) : (W)0;
  }
  __syncthreads();
  if (tid < (1 << inner)) {
    W e = 0;
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      if (u >= B || !((tid >> u) & 1)) continue;
      W row = qin[u][u];
#pragma unroll
      for (int w = u + 1; w < 6; ++w)
        if (w < B && ((tid >> w) & 1)) row += qin[u][w];
      e += row;
    }
    if (wide) ((double*)v.ei)[(int64_t)b * 64 + tid] = (double)e;  // exact: |e| <= sum |Q|
    else ((W*)v.ei)[(int64_t)b * 64 + tid] = e;
  }
  if (tid == 0) {
    const double sa = red_a[0];
    I->sumabs = sa;
    I->hscale = 1.0;
    I->hmargin = 0.0;
    I->wide = wide ? 1 : 0;
    if constexpr (std::is_same_v<E, int32_t>) {
      I->big = sa + 1.0;
      I->eps = 0.0;
      if (wide) {
        if (sa > kWideSumLimit) I->status = kErrRange;  // cannot happen for n <= 63; kept as a guard
        set_half_screen(I, red_r[0], sa);
      } else {
        // int16 screen: C', Tb, Ta and their sums are partial sums of the
        // inner rows, exact int16 values when R_I <= 32767
        I->hscale = red_r[0] <= (double)kInt16Limit ? 1.0 : 0.0;
      }
    } else if constexpr (std::is_integral_v<Qin>) {
      // integer Q on the float64 walk: exact below kWideSumLimit
      I->big = sa + 1.0;
      I->eps = 0.0;
      if (sa > kWideSumLimit) I->status = kErrRange;
    } else if constexpr (std::is_same_v<E, double>) {
      // float64 walk: C', T', the step constants and the running Dp are sums
      // of at most n + 2^14 + n^2 roundings of magnitude <= u sum|Q|
      // (u = 2^-53), well inside 2^-36 sum|Q|; exact for integer-valued Q
      // with sum |Q| <= 2^50.
      I->big = sa * (1.0 + 1e-9) + 1.0;
      I->eps = 0x1p-36 * sa;
      if (!red_frac[0] && sa <= kWideSumLimit) {
        // exact: integer thresholds keep every offset and key an integer
        I->eps = 0.0;
        I->big = sa + 1.0;
      }
      if (red_bad[0]) I->status = kErrNonfinite;
    } else {
      I->big = sa * (1.0 + 1e-6) + 1.0;
      // |f32 table value - exact| <= 2u * R_I with u = 2^-24 (C', T' and their sum
      // are partial sums of the inner rows); the rest is float64 rounding.
      // The running offset Dp and the replay keys are float64 (the bound of
      // the float64 walk below).
      I->eps = 3.0 * 0x1p-24 * red_r[0] + 0x1p-36 * sa;
      // Integer-valued float Q with sum |Q| <= 2^24: every table value, sum and
      // key is an integer below 2^24 in magnitude, exact in float32 and float64,
      // so the walk is exact (eps = 0) and ties are resolved like the int path.
      // The threshold bound is then an integer as well: a fractional
      // threshold would round the float64 offset Dp = thr - E_P (and the replay
      // keys taken from it) by a lane-dependent amount, and equal energies
      // would no longer compare equal.
      if (!red_frac[0] && sa <= 16777216.0) {
        I->eps = 0.0;
        I->big = sa + 1.0;
      }
      if (red_bad[0]) I->status = kErrNonfinite;
    }
    if constexpr (!std::is_same_v<E, int32_t>) set_half_screen(I, red_r[0], sa);
  }
}

// Lane table: for each lane value l (the L lane bits at positions B+no..),
// record [0] = the lane bits' own energy, [1+u] = sum_{set lane bits a}
// S(u, a) for inner bits u, [8+k] = sum_{set lane bits a} S(B+k, a) for outer
// bits k.
template <class W>
__device__ void lanes_role(const Views& v, int b, int l, W* st) {
  // One wave: the entries of Q the records need are staged in LDS by
  // independent loads (three per lane), so their latencies overlap; lane l
  // then sums them for its set bits, in the order of a loop over the bits.
  const Inst* I = &v.inst[b];
  W* lt = (W*)v.lt + ((int64_t)b * 64 + l) * kLaneRec;
  W rec[kLaneRec];
  for (int i = 0; i < kLaneRec; ++i) rec[i] = 0;
  if (I->status == 0) {
    const int L = I->L, B = I->B, no = I->no, pos0 = B + no, nm = v.nmax;
    const W* qs = (const W*)v.qs + (int64_t)b * nm * nm;
    // column a of lane bit a (ra = pos0 + a): [0] Q(ra, ra), [1 + a2]
    // Q(ra, pos0 + a2), [7 + u] Q(u, ra) for inner u, [13 + k] Q(B + k, ra)
    // for outer k
    constexpr int kCol = 13 + kMaxOuter;
    static_assert(6 * kCol <= 3 * kWave, "three staged entries per lane");
    W q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int e = l + kWave * d, a = e / kCol, f = e % kCol, ra = pos0 + a;
      int row = -1, col = 0;
      if (a < L) {
        if (f == 0) row = ra, col = ra;
        else if (f < 7) { if (f - 1 > a && f - 1 < L) row = ra, col = pos0 + f - 1; }
        else if (f < 13) { if (f - 7 < B) row = f - 7, col = ra; }
        else if (f - 13 < no) row = B + f - 13, col = ra;
      }
      q[d] = row >= 0 ? qs[(int64_t)row * nm + col] : (W)0;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (l + kWave * d < 6 * kCol) st[l + kWave * d] = q[d];
    __builtin_amdgcn_wave_barrier();
    // fixed trip counts, so that rec stays in registers
    static_assert(8 + kMaxOuter <= kLaneRec, "the record holds every outer field");
    if (l < (1 << L)) {
      for (int a = 0; a < L; ++a) {
        if (!((l >> a) & 1)) continue;
        const W* c = st + a * kCol;
        rec[0] += c[0];
        for (int a2 = a + 1; a2 < L; ++a2)
          if ((l >> a2) & 1) rec[0] += c[1 + a2];
#pragma unroll
        for (int u = 0; u < 6; ++u)
          if (u < B) rec[1 + u] += c[7 + u];
#pragma unroll
        for (int k = 0; k < kMaxOuter; ++k)
          if (k < no) rec[8 + k] += c[13 + k];
      }
    }
  }
  for (int i = 0; i < kLaneRec; ++i) lt[i] = rec[i];
}

// SplitMix64 output function (Steele, Lea, Flood 2014), used as a hash.
__device__ uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Local field h_i(x) = sum_{j != i} S_ij x_j of row i (zero diagonal, row
// stride np, zero padding), four independent partial sums.
template <class T>
__device__ __forceinline__ T field(const T* row, int np, uint64_t x) {
  T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (int j = 0; j < np; j += 4) {
    a0 += ((x >> j) & 1) ? row[j] : (T)0;
    a1 += ((x >> (j + 1)) & 1) ? row[j + 1] : (T)0;
    a2 += ((x >> (j + 2)) & 1) ? row[j + 2] : (T)0;
    a3 += ((x >> (j + 3)) & 1) ? row[j + 3] : (T)0;
  }
  return (a0 + a1) + (a2 + a3);
}

constexpr int kSeedThreads = 256;  // a single instance's seed: four waves of descents

// A-priori threshold for instance b.  Its waves (one or four) run
// `seed_sweeps` steepest one-flip descents between them, from their own
// starts (wave 0's first from x = 0): lane j holds the field
// h_j = sum_i S_ij x_i of bit j in float32, every step flips the bit with the
// most negative change (a wave minimum) and moves the fields by one row of S,
// until no flip lowers f or 4n steps have been taken.  The best local minimum
// x*, its n one-flip and n(n-1)/2 two-flip neighbours are distinct states, so
// the K'-th smallest of their values bounds the instance's K'-th smallest
// value from above.  Published with the float filter's error margin, the
// bound discards nothing the walk would keep; it only spares each wave the
// replays of its cold start.  A prefix-range solve keeps its top seed_fix
// bits at the range's first prefix and descends over the free bits only, so
// that x* and its free-bit neighbours lie in the range and bound the range's
// K'-th smallest value.
//
// With S the symmetric off-diagonal part and d the diagonal,
//   f(x) = sum_i x_i (d_i + h_i(x) / 2),  f(x ^ e_i) = f(x) + (1 - 2 x_i)(d_i + h_i(x)),
// so lane i evaluates one field of x* and the wave sums: O(n) per lane; a
// two-flip value adds s_i s_j S_ij (s = 1 - 2x) to the two one-flip changes.
template <class W>
__device__ void seed_role(const Views& v, int b, unsigned char* seed_lds) {
  __shared__ float best_f[kSeedThreads / kWave];
  __shared__ uint64_t best_x[kSeedThreads / kWave];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nt = blockDim.x, nwv = nt >> 6;
  const Inst* I = &v.inst[b];
  if (I->status != 0) return;  // uniform over the block
  const int n = I->n, kp = I->kprime, nm = v.nmax;
  const int fix = I->seed_fix, nf = n - fix;  // free (searched) bits: [0, nf)
  const int np = (n + 3) & ~3;
  // exact (W) and float32 copies of S with zero diagonal and padded rows, and
  // d; the block's threads fill them with several independent loads each
  W* sw = (W*)seed_lds;
  W* dw = sw + np * np;
  float* sf = (float*)(dw + np);
  float* df = sf + np * np;
  const W* qg = (const W*)v.qs + (int64_t)b * nm * nm;
  constexpr int kU = 4;
  for (int e0 = tid; e0 < np * np; e0 += kU * nt) {
    W q[kU];
#pragma unroll
    for (int d = 0; d < kU; ++d) {
      const int e = e0 + d * nt;
      const int i = e / np, j = e % np;
      q[d] = (e < np * np && i < n && j < n && i != j) ? qg[(int64_t)i * nm + j] : (W)0;
    }
#pragma unroll
    for (int d = 0; d < kU; ++d) {
      const int e = e0 + d * nt;
      if (e < np * np) {
        sw[e] = q[d];
        sf[e] = (float)q[d];
      }
    }
  }
  for (int i = tid; i < np; i += nt) {
    dw[i] = i < n ? qg[(int64_t)i * nm + i] : (W)0;
    df[i] = (float)dw[i];
  }
  __syncthreads();
  const uint64_t free = nf >= 64 ? ~0ull : ((1ull << nf) - 1);
  const uint64_t base = fix > 0 ? ((uint64_t)I->local_off >> (I->tb - fix)) << nf : 0;
  // descents in float32 (any states back the bound, so neither exact deltas
  // nor convergence matter here); lanes j >= nf never flip
  const int runs = (v.seed_sweeps + nwv - 1) / nwv;  // the instance's descents, spread over its waves
  const float dj = lane < n ? df[lane] : 0.f;
  float bf = __builtin_inff();
  uint64_t bx = base;
  for (int run = 0; run < runs; ++run) {
    const int id = w * runs + run;
    uint64_t x = base | (id == 0 ? 0 : (mix64(((uint64_t)b << 8) | (uint64_t)id) & free));
    float h = 0.f;  // h_j of lane j < n
    if (lane < n)
      for (int i = 0; i < n; ++i)
        if ((x >> i) & 1) h += sf[i * np + lane];
    for (int step = 0; step < 4 * n; ++step) {
      const float g = dj + h;
      const float dlt = lane < nf ? (((x >> lane) & 1) ? -g : g) : __builtin_inff();
      const float m = wave_min_f32(dlt);
      if (!(m < 0.f)) break;
      const int j = __builtin_ctzll(ballot(dlt == m));
      x ^= 1ull << j;
      if (lane < n) h += ((x >> j) & 1) ? sf[j * np + lane] : -sf[j * np + lane];
    }
    // f(x) = sum_j x_j (d_j + h_j / 2); the wave's best, ties to the lower x
    const float fx = wave_sum_f32(((x >> lane) & 1) && lane < n ? dj + 0.5f * h : 0.f);
    if (fx < bf || (fx == bf && x < bx)) {
      bf = fx;
      bx = x;
    }
  }
  if (lane == 0) {
    best_f[w] = bf;
    best_x[w] = bx;
  }
  __syncthreads();
  if (w != 0) return;
  int bw = 0;
  for (int o = 1; o < nwv; ++o)
    if (best_f[o] < best_f[bw]) bw = o;
  const uint64_t xs = uniform_u64(best_x[bw]);
  // exact values: lane i < n evaluates field i of x*
  W gi = 0, term = 0;
  if (lane < n) {
    gi = dw[lane] + field(sw + lane * np, np, xs);  // d_i + h_i(x*)
    if ((xs >> lane) & 1) term = dw[lane] + gi;      // 2 x_i (d_i + h_i / 2)
  }
  W tot = term;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
  if constexpr (std::is_same_v<W, double>) tot = uniform_f64(tot) * 0.5;
  else tot = (W)uniform_u64((uint64_t)tot) / 2;  // even: 2 sum_i x_i d_i + 2 sum_{i<j} S_ij x_i x_j
  // x* and its one-flip neighbours (D_i = f(x* ^ e_i) - f(x*)), sorted: the
  // first K' form the candidate list
  const W si = ((xs >> lane) & 1) ? (W)-1 : (W)1;
  const W Di = lane < nf ? si * gi : (W)0;
  double key = __builtin_inf();
  uint64_t mask = ~0ull;
  if (lane < nf) {
    mask = xs ^ (1ull << lane);
    key = (double)(tot + Di);
  } else if (lane == nf) {
    mask = xs;
    key = (double)tot;
  }
  wave_sort(key, mask, lane);
  double lkey = lane < kp ? key : __builtin_inf();
  uint64_t lmask = lane < kp ? mask : ~0ull;
  // two-flip neighbours x* ^ e_i ^ e_j (lane i < j < nf):
  //   f = f(x*) + D_i + D_j + s_i s_j S_ij,  s = 1 - 2 x*
  // so every K' up to 64 is backed once nf >= 11
  for (int j = 1; j < nf; ++j) {
    W Dj, sj;
    if constexpr (std::is_same_v<W, double>) Dj = readlane_f64(Di, j);
    else Dj = readlane_i64(Di, j);
    sj = ((xs >> j) & 1) ? (W)-1 : (W)1;
    const bool ok = lane < j;
    const W sij = sw[(ok ? lane : 0) * np + j];
    const double ck = ok ? (double)(tot + Di + Dj + si * sj * sij) : __builtin_inf();
    const uint64_t cm = xs ^ (1ull << lane) ^ (1ull << j);
    double tk = readlane_f64(lkey, kp - 1);
    uint64_t tm = readlane_u64(lmask, kp - 1);
    uint64_t bal = ballot(ok && before(ck, cm, tk, tm));
    while (bal) {
      const int src = __builtin_ctzll(bal);
      bal &= bal - 1;
      const double k2 = readlane_f64(ck, src);
      const uint64_t m2 = readlane_u64(cm, src);
      if (before(k2, m2, tk, tm)) {
        list_insert(lkey, lmask, k2, m2, kp, lane);
        tk = readlane_f64(lkey, kp - 1);
        tm = readlane_u64(lmask, kp - 1);
      }
    }
  }
  const double vk = readlane_f64(lkey, kp - 1);
  if (lane == 0 && vk < __builtin_inf()) {
    // float: the walk's filter error (eps) plus float64 rounding of the sums
    // here.  Exact instances (eps = 0: integer data whose sums stay below
    // 2^53) publish the value itself, an integer, so that the walk's offsets
    // and replay keys stay exact and equal energies compare equal.
    const double margin = (std::is_same_v<W, double> && I->eps > 0.0) ? I->eps + 1e-12 * I->sumabs : 0.0;
    v.gthr[b] = enc_key(vk + margin);
  }
}

// kWideI32: an int32 instance beyond the int32 walk's range (float64 W, float16
// rows in the int32 layout's 256-byte step slots, whatever the screen knob).
template <class W, class E, bool kWideI32 = false>
__device__ void tables_role(const Views& v, int b, int chunk, int inner, unsigned char* lds) {
  // chunk: blockDim.x consecutive steps of instance b.  The entries the step
  // scalars need -- S(u, B+l) for inner u and S(B+l, B+l2) for outer l, l2 --
  // are staged in LDS.  A wave takes 64 consecutive steps: lane i computes the
  // scalars of step s0 + i, parks H in LDS, and the wave then writes the 64
  // table rows one coalesced row at a time.
  W(*hs)[6][kWave] = (W(*)[6][kWave])lds;  // [waves][6][64]
  W* qo = (W*)(lds + sizeof(W) * (blockDim.x / kWave) * 6 * kWave);
  const Inst* I = &v.inst[b];
  if (I->status != 0) return;  // the walks skip such instances
  const int B = I->B, no = I->no, nm = v.nmax;
  const int64_t steps = int64_t(1) << no;
  const int64_t c0 = (int64_t)chunk * blockDim.x;
  if (c0 >= steps) return;
  const W* qs = (const W*)v.qs + (int64_t)b * nm * nm;
  // row r < 6: inner row u = r; row 6 + l: outer row B + l; column l2: B + l2;
  // up to (6 + kMaxOuter) kMaxOuter entries, three loads per thread of a
  // 64-thread block in flight together
  const int nq = (6 + no) * no;
  for (int e0 = threadIdx.x; e0 < nq; e0 += 3 * blockDim.x) {
    W q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int e = e0 + d * blockDim.x, r = e / no, l2 = e % no;
      q[d] = (e >= nq || (r < 6 && r >= B)) ? (W)0 : qs[(int64_t)(r < 6 ? r : B + r - 6) * nm + B + l2];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (e0 + d * blockDim.x < nq) qo[e0 + d * blockDim.x] = q[d];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t s0 = c0 + (int64_t)w * kWave;  // the wave's first step
  if (s0 >= steps) return;
  const int width = 1 << inner, per = width / 16;
  const int64_t t = s0 + lane;
  W H[6] = {0, 0, 0, 0, 0, 0};
  W eo = 0;
  if (t < steps) {
    const uint64_t o = gray((uint64_t)t);
    for (int l = 0; l < no; ++l) {
      if (!((o >> l) & 1)) continue;
      W row = qo[(6 + l) * no + l];
      for (int l2 = l + 1; l2 < no; ++l2)
        if ((o >> l2) & 1) row += qo[(6 + l) * no + l2];
      eo += row;
#pragma unroll
      for (int u = 0; u < 6; ++u) H[u] += qo[u * no + l];  // zero rows for u >= B
    }
    const int64_t s = I->tab_off + t;
    v.eod[s] = (double)eo;
    StepRec* r = &v.rec[s];
    r->eo = (double)eo;
#pragma unroll
    for (int u = 0; u < 6; ++u) r->h[u] = (double)H[u];
    // -E_O as int32: read by the int32 walks only (|E_O| <= sum |Q| <= 2^28 there)
    const int32_t neo = std::is_same_v<E, int32_t> ? (int32_t)(-eo) : 0;
    v.eoi[s] = neo;
    r->neo = neo;
    r->pad = 0;
    if constexpr (std::is_same_v<E, int32_t>) {
      if (v.h16 && I->hscale != 0.0) {
        // the int16 screen's row: exact Tb / Ta from the linear split of T'
        auto h16 = [](W x) { return (uint32_t)(uint16_t)(int16_t)x; };
        HalfRow hr;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          W lo = 0;  // Tb(2k); Tb(2k + 1) adds H_0
#pragma unroll
          for (int u = 1; u < 4; ++u) {
            if (((2 * k) >> u) & 1) lo += H[u];
          }
          hr.tb[k] = h16(lo) | (h16(lo + H[0]) << 16);
        }
        hr.ta[0] = h16(0) | (h16(H[5]) << 16);
        hr.ta[1] = h16(H[4]) | (h16(H[4] + H[5]) << 16);
        hr.neo = (int32_t)(-eo);
        hr.pad0 = hr.pad1[0] = hr.pad1[1] = 0;
        hr.tau = 0.0;
        ((HalfRow*)v.tab)[s * kInt16RowStride] = hr;
      }
    }
    if constexpr (!std::is_same_v<E, int32_t>) {
      if (kWideI32 || v.h16) {
        // the half screen's row: Tb / Ta from the linear split of T'
        const double hs = I->hscale;
        auto h16 = [&](double x) { return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(float)(x * hs)); };
        HalfRow hr;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          double lo = 0, hi = 0;  // Tb(2k), Tb(2k + 1)
#pragma unroll
          for (int u = 1; u < 4; ++u) {
            if (((2 * k) >> u) & 1) lo += (double)H[u];
          }
          hi = lo + (double)H[0];
          hr.tb[k] = h16(lo) | (h16(hi) << 16);
        }
        const double ta[4] = {0.0, (double)H[4], (double)H[5], (double)H[4] + (double)H[5]};
        hr.ta[0] = h16(ta[0]) | (h16(ta[2]) << 16);
        hr.ta[1] = h16(ta[1]) | (h16(ta[3]) << 16);
        hr.neo = 0;
        hr.pad0 = hr.pad1[0] = hr.pad1[1] = 0;
        hr.tau = (double)eo * hs - I->hmargin;
        ((HalfRow*)v.tab)[kWideI32 ? s * kInt16RowStride : s] = hr;
      }
    }
  }
  if constexpr (!std::is_same_v<E, int32_t>) {
    if (kWideI32 || v.h16) return;  // the half screen reads HalfRow rows only
  }
  if constexpr (std::is_same_v<E, int32_t>) {
    if (v.h16 && I->hscale != 0.0) return;  // the int16 screen reads HalfRow rows only
  }
#pragma unroll
  for (int u = 0; u < 6; ++u) hs[w][u][lane] = H[u];
  __builtin_amdgcn_wave_barrier();
  E* tab = (E*)v.tab + I->tab_off * width;
  const int nst = (int)(steps - s0 < kWave ? steps - s0 : kWave);
#pragma unroll 4
  for (int k = 0; k < nst; ++k) {
    // H_u is zero for u >= B, so summing every set lane bit is the same sum
    W tj = 0;
#pragma unroll
    for (int u = 0; u < 6; ++u)
      if ((lane >> u) & 1) tj += hs[w][u][k];
    if (lane < width) tab[(s0 + k) * width + (lane & 15) * per + (lane >> 4)] = (E)tj;
  }
}

// The per-instance inputs of a walk, in one launch: blockIdx.x is the
// instance; blockIdx.y = 0 the threshold seed (when seed_on), 1 the lane
// table, 2 + c the step tables of chunk c.  The three only read what
// prep_inst wrote, so their latencies overlap.
template <class W, class E, bool kWideI32>
__device__ void prep_walk_roles(const Views& v, int b, int role, int inner, int seed_on, unsigned char* lds) {
  if (role == 0) {
    if (seed_on) seed_role<W>(v, b, lds);
  } else if (role == 1) {
    if (threadIdx.x < kWave) lanes_role<W>(v, b, threadIdx.x, (W*)lds);
  } else {
    tables_role<W, E, kWideI32>(v, b, role - 2, inner, lds);
  }
}

template <class W, class E>
__global__ void __launch_bounds__(kSeedThreads) prep_walk_kernel(Views v, int inner, int seed_on) {
  extern __shared__ __attribute__((aligned(16))) unsigned char prep_lds[];
  const int b = blockIdx.x, role = blockIdx.y;
  if constexpr (std::is_same_v<E, int32_t>) {
    if (v.inst[b].wide) {  // float64 tables, half-screen rows (uniform over the block)
      prep_walk_roles<double, float, true>(v, b, role, inner, seed_on, prep_lds);
      return;
    }
  }
  prep_walk_roles<W, E, false>(v, b, role, inner, seed_on, prep_lds);
}

}  // namespace

hipError_t launch_plan(const Views& v, const int32_t* ns, int n_single, const float* beta, const PlanParams& pp,
                       hipStream_t s) {
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, s, v, ns, n_single, beta, pp);
  return hipGetLastError();
}

hipError_t launch_prep_inst(const Views& v, const void* q, int64_t ldq, int64_t stride, int dt, int inner,
                            hipStream_t s) {
  const dim3 g(v.batch), blk(256);
  switch (dt) {
    case kDtI32:
      hipLaunchKernelGGL((prep_inst_kernel<int32_t, int64_t, int32_t>), g, blk, 0, s, v, (const int32_t*)q, ldq,
                         stride, inner);
      break;
    case kDtF64:
      hipLaunchKernelGGL((prep_inst_kernel<double, double, double>), g, blk, 0, s, v, (const double*)q, ldq,
                         stride, inner);
      break;
    case kDtI64:
      hipLaunchKernelGGL((prep_inst_kernel<int64_t, double, double>), g, blk, 0, s, v, (const int64_t*)q, ldq,
                         stride, inner);
      break;
    default:
      hipLaunchKernelGGL((prep_inst_kernel<float, double, float>), g, blk, 0, s, v, (const float*)q, ldq, stride,
                         inner);
  }
  return hipGetLastError();
}

hipError_t launch_prep_walk(const Views& v, int dt, int inner, int64_t steps_bound, bool seed, hipStream_t s) {
  // a single instance: 256 threads (four waves of seed descents, 256 steps
  // per table block); a batch: one wave per block
  const int T = v.batch == 1 ? kSeedThreads : kWave;
  const int64_t per_inst = (steps_bound + v.batch - 1) / v.batch;  // steps of one instance, bound
  const int64_t chunks = (per_inst + T - 1) / T > 0 ? (per_inst + T - 1) / T : 1;
  const dim3 grid((unsigned)v.batch, (unsigned)(2 + chunks));
  const bool seed_on = seed && v.seed_sweeps > 0;
  // dynamic LDS: the seed's padded n x n (8-byte exact + float32 copies) and
  // diagonal, or the tables' staging, whichever is larger
  const size_t np = (size_t)((v.nmax + 3) & ~3);
  const size_t seed_bytes = seed_on ? (sizeof(double) + sizeof(float)) * (np * np + np) : 0;
  const size_t tab_bytes = sizeof(double) * ((size_t)(T / kWave) * 6 * kWave + (6 + kMaxOuter) * kMaxOuter);
  const size_t lds = seed_bytes > tab_bytes ? seed_bytes : tab_bytes;
  if (dt == kDtI32)
    hipLaunchKernelGGL((prep_walk_kernel<int64_t, int32_t>), grid, dim3(T), lds, s, v, inner, (int)seed_on);
  else if (dt_wide(dt))
    hipLaunchKernelGGL((prep_walk_kernel<double, double>), grid, dim3(T), lds, s, v, inner, (int)seed_on);
  else
    hipLaunchKernelGGL((prep_walk_kernel<double, float>), grid, dim3(T), lds, s, v, inner, (int)seed_on);
  return hipGetLastError();
}

}  // namespace qbf
