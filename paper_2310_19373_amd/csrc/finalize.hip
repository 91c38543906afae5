// Merge of the flushed candidate lists, rescoring and the float certificate.
//
// One block per instance (W waves).  Each wave scans a share of the instance's
// flushed lists, keeping its own sorted top-K' (filtered by the instance's
// published threshold, which bounds the final K'-th key from above; a chunk
// with many qualifying entries is sorted and merged by bitonic networks, a
// few are inserted one by one); the waves' lists are merged pairwise through
// LDS.  Every candidate's energy is then recomputed from the input Q in a
// fixed order -- i ascending; for each set bit i the row term starts at Q_ii
// and adds Q_ij for set j > i in ascending j; row terms summed in ascending i
// -- in float64 (float Q) or int64 (int Q), spread over the waves (one lane per
// row) when there are four or more, else one lane per candidate.  Wave 0 sorts
// by (energy, mask), writes the k best and, for float Q, checks the
// certificate: every state outside the candidate set has an exact value of at
// least thr - eps, where thr is the K'-th candidate key, so the selection is
// exact when thr - eps exceeds the k-th rescored energy.
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"
#include "wave.hpp"

namespace qbf {

namespace {

__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ int64_t add_rn(int64_t a, int64_t b) { return a + b; }

// Row term of the canonical order: Q_ii, then Q_ij for set j > i in ascending
// j, in En.  A row's entries are read eight at a time ahead of its additions,
// whose order is unchanged.
template <class T, class En>
__device__ __forceinline__ En row_term(const T* Q, int ldq, int n, int i, uint64_t m) {
  En row = (En)Q[i * ldq + i];
  for (int j0 = i + 1; j0 < n; j0 += 8) {
    T q[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) q[d] = j0 + d < n ? Q[i * ldq + j0 + d] : (T)0;
#pragma unroll
    for (int d = 0; d < 8; ++d)
      if (j0 + d < n && ((m >> (j0 + d)) & 1)) row = add_rn(row, (En)q[d]);
  }
  return row;
}

// Canonical-order energy: row terms of the set rows added in ascending i, in
// En (float64 or int64).
template <class T, class En>
__device__ __forceinline__ En canonical_energy(const T* Q, int ldq, int n, uint64_t m) {
  En tot = 0;
  for (int i = 0; i < n; ++i)
    if ((m >> i) & 1) tot = add_rn(tot, row_term<T, En>(Q, ldq, n, i, m));
  return tot;
}

// Bitonic merge of two wave lists, each ascending by (key, mask) over the 64
// lanes, into the 64 smallest entries of their union, ascending.
__device__ __forceinline__ void merge64(double& ak, uint64_t& am, double bk, uint64_t bm, int lane) {
  const double rk = __shfl(bk, kWave - 1 - lane);
  const uint64_t rm = __shfl(bm, kWave - 1 - lane);
  if (before(rk, rm, ak, am)) {  // lane-wise minimum of a and reversed b: bitonic
    ak = rk;
    am = rm;
  }
#pragma unroll
  for (int j = kWave / 2; j > 0; j >>= 1) {
    const double pk = __shfl_xor(ak, j);
    const uint64_t pm = __shfl_xor(am, j);
    const bool lower = (lane & j) == 0;
    if (lower ? before(pk, pm, ak, am) : before(ak, am, pk, pm)) {
      ak = pk;
      am = pm;
    }
  }
}

// Output type and sentinel per input type.
template <class Qin>
struct Rescore {
  using En = std::conditional_t<std::is_floating_point_v<Qin>, double, int64_t>;
  __device__ static En sentinel() {
    if constexpr (std::is_floating_point_v<Qin>) return __builtin_inf();
    else return INT64_MAX;
  }
  __device__ static En energy(const Qin* Q, int ldq, int n, uint64_t m) {
    return canonical_energy<Qin, En>(Q, ldq, n, m);
  }
};

__device__ __forceinline__ int64_t readlane_en(int64_t v, int l) { return readlane_i64(v, l); }
__device__ __forceinline__ double readlane_en(double v, int l) { return readlane_f64(v, l); }

constexpr int kMaxFinWaves = 16;

template <class Qin>
__global__ void __launch_bounds__(1024) finalize_topk_kernel(Views v, const Qin* q, int64_t ldq, int64_t stride,
                                                             int k, typename Rescore<Qin>::En* energies,
                                                             uint64_t* masks, int32_t* status) {
  using En = typename Rescore<Qin>::En;
  // LDS sized by the launch (launch_finalize_topk): the waves' lists, the
  // rescored energies and the instance's n x n block of Q (row stride
  // n <= nmax), so that a batch's one-wave blocks are not held to a few per CU
  extern __shared__ __attribute__((aligned(16))) unsigned char fin_lds[];
  const int b = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double(*const sk)[kWave] = (double(*)[kWave])fin_lds;
  uint64_t(*const sm)[kWave] = (uint64_t(*)[kWave])(fin_lds + (size_t)nw * kWave * sizeof(double));
  En* const se = (En*)(fin_lds + (size_t)nw * kWave * (sizeof(double) + sizeof(uint64_t)));
  Qin* const sq = (Qin*)(se + kMaxKPrime);
  const Inst* I = &v.inst[b];
  const int kp = I->kprime;
  const int32_t st0 = I->status;
  double lkey = __builtin_inf();
  uint64_t lmask = ~0ull;
  if (st0 == 0) {
    const int64_t cnt = min<int64_t>((int64_t)v.flushcnt[b], I->slot_cap);
    const int64_t total = cnt * kp;
    const Slot* sl = v.slots + I->slot_off * kp;
    double thr = fmin(dec_key(v.gthr[b]), I->big);
    for (int64_t base = (int64_t)w * kWave; base < total; base += (int64_t)nw * kWave) {
      const int64_t e = base + lane;
      double key = __builtin_inf();
      uint64_t m = ~0ull;
      if (e < total) {
        key = sl[e].key;
        m = sl[e].mask;
      }
      uint64_t bal = ballot(key <= thr);
      if (__popcll(bal) > 8) {
        // many candidates: sort them and merge (two bitonic networks) rather
        // than insert one at a time
        const bool c = key <= thr;
        double ck = c ? key : __builtin_inf();
        uint64_t cm = c ? m : ~0ull;
        wave_sort(ck, cm, lane);
        merge64(lkey, lmask, ck, cm, lane);
        if (lane >= kp) {
          lkey = __builtin_inf();
          lmask = ~0ull;
        }
        const double lt = readlane_f64(lkey, kp - 1);
        if (lt < thr) thr = lt;
        continue;
      }
      while (bal) {
        const int src = __builtin_ctzll(bal);
        bal &= bal - 1;
        const double ck = readlane_f64(key, src);
        if (ck <= thr && list_insert(lkey, lmask, ck, readlane_u64(m, src), kp, lane)) {
          const double lt = readlane_f64(lkey, kp - 1);
          if (lt < thr) thr = lt;
        }
      }
    }
  }
  sk[w][lane] = lkey;
  sm[w][lane] = lmask;
  const int n = I->n;
  if (st0 == 0) {
    const Qin* Qb = q + (int64_t)b * stride;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) sq[e] = Qb[(int64_t)(e / n) * ldq + e % n];
  }
  __syncthreads();
  // the waves' lists, merged pairwise in log2(waves) rounds; sk[0] ends with
  // the K' best
  for (int r = 1; r < nw; r <<= 1) {
    if ((w & (2 * r - 1)) == 0 && w + r < nw) {
      merge64(lkey, lmask, sk[w + r][lane], sm[w + r][lane], lane);
      if (lane >= kp) {
        lkey = __builtin_inf();
        lmask = ~0ull;
      }
      sk[w][lane] = lkey;
      sm[w][lane] = lmask;
    }
    __syncthreads();
  }
  En en = Rescore<Qin>::sentinel();
  uint64_t m = ~0ull;
  if (nw >= 4) {
    // rescoring spread over the waves: wave w takes candidates w, w + nw, ...;
    // lane i computes row i's term and the wave adds the set rows' terms in
    // ascending i (the canonical order)
    for (int c = w; c < kp; c += nw) {
      const double ckey = sk[0][c];
      const uint64_t cm = sm[0][c];
      En tot = Rescore<Qin>::sentinel();
      if (st0 == 0 && ckey < __builtin_inf()) {
        En r = 0;
        if (lane < n && ((cm >> lane) & 1)) r = row_term<Qin, En>(sq, n, n, lane, cm);
        tot = 0;
        for (int i = 0; i < n; ++i)
          if ((cm >> i) & 1) tot = add_rn(tot, readlane_en(r, i));
      }
      if (lane == 0) se[c] = tot;
    }
    __syncthreads();
    if (w != 0) return;
    if (st0 == 0 && lane < kp && lkey < __builtin_inf()) {
      m = lmask;
      en = se[lane];
    }
  } else {
    if (w != 0) return;
    if (st0 == 0 && lane < kp && lkey < __builtin_inf()) {
      m = lmask;
      en = Rescore<Qin>::energy(sq, n, n, m);
    }
  }
  int32_t st = st0;
  if (st == 0 && (int64_t)v.flushcnt[b] > I->slot_cap) st = kErrOverflow;
  wave_sort(en, m, lane);
  if constexpr (std::is_floating_point_v<Qin>) {
    const double thr_m = readlane_f64(lkey, kp - 1);
    const double ek = readlane_en(en, k - 1);
    if (st == 0 && I->eps > 0.0 && thr_m < __builtin_inf() && !(thr_m - I->eps > ek)) st = kErrUncertain;
  }
  if (lane < k) {
    const bool ok = (st == 0 || st == kErrUncertain);
    energies[(int64_t)b * k + lane] = ok ? en : Rescore<Qin>::sentinel();
    masks[(int64_t)b * k + lane] = ok ? m : ~0ull;
  }
  if (lane == 0) status[b] = st;
}

// Merge of `count` lists of k_in (energy, mask) entries -- results of solves
// over disjoint prefix ranges of one instance -- into the k best by (energy,
// mask).  One wave: entries stream through 64 at a time, and those that beat
// the current k-th are inserted into the wave's sorted list.  Energies pass
// through float64 keys, exact for the int paths' |E| <= 2^50 as well.
template <class En>
__global__ void __launch_bounds__(64) merge_topk_kernel(int count, int k_in, const En* ein, const uint64_t* min_,
                                                        int k, En* eout, uint64_t* mout) {
  const int lane = threadIdx.x;
  double lkey = __builtin_inf();
  uint64_t lmask = ~0ull;
  const int64_t total = (int64_t)count * k_in;
  for (int64_t base = 0; base < total; base += kWave) {
    const int64_t e = base + lane;
    double key = __builtin_inf();
    uint64_t m = ~0ull;
    if (e < total) {
      const En x = ein[e];
      if (x != Rescore<En>::sentinel()) {
        key = (double)x;
        m = min_[e];
      }
    }
    const double tk = readlane_f64(lkey, k - 1);
    const uint64_t tm = readlane_u64(lmask, k - 1);
    uint64_t bal = ballot(key < __builtin_inf() && before(key, m, tk, tm));
    while (bal) {
      const int src = __builtin_ctzll(bal);
      bal &= bal - 1;
      list_insert(lkey, lmask, readlane_f64(key, src), readlane_u64(m, src), k, lane);
    }
  }
  if (lane < k) {
    const bool fin = lkey < __builtin_inf();
    eout[lane] = fin ? (En)lkey : Rescore<En>::sentinel();
    mout[lane] = fin ? lmask : ~0ull;
  }
}

}  // namespace

hipError_t launch_finalize_topk(const Views& v, const void* q, int64_t ldq, int64_t stride, int dt, int k,
                                void* energies, uint64_t* masks, int32_t* status, int waves_per_inst,
                                hipStream_t s) {
  const int w = max(1, min(kMaxFinWaves, waves_per_inst));
  const dim3 g(v.batch), blk(64 * w);
  // bytes of fin_lds: w lists of 64 (key, mask), kMaxKPrime energies, nmax^2 entries of Q
  auto lds = [&](size_t qbytes) {
    return (size_t)w * kWave * (sizeof(double) + sizeof(uint64_t)) + kMaxKPrime * 8 + (size_t)v.nmax * v.nmax * qbytes;
  };
  switch (dt) {
    case kDtI32:
      hipLaunchKernelGGL(finalize_topk_kernel<int32_t>, g, blk, lds(4), s, v, (const int32_t*)q, ldq, stride, k,
                         (int64_t*)energies, masks, status);
      break;
    case kDtF64:
      hipLaunchKernelGGL(finalize_topk_kernel<double>, g, blk, lds(8), s, v, (const double*)q, ldq, stride, k,
                         (double*)energies, masks, status);
      break;
    case kDtI64:
      hipLaunchKernelGGL(finalize_topk_kernel<int64_t>, g, blk, lds(8), s, v, (const int64_t*)q, ldq, stride, k,
                         (int64_t*)energies, masks, status);
      break;
    default:
      hipLaunchKernelGGL(finalize_topk_kernel<float>, g, blk, lds(4), s, v, (const float*)q, ldq, stride, k,
                         (double*)energies, masks, status);
  }
  return hipGetLastError();
}

}  // namespace qbf

namespace qbf {

hipError_t launch_merge_topk(int count, int k_in, const void* ein, const uint64_t* min, int dt, int k, void* eout,
                             uint64_t* mout, hipStream_t s) {
  if (dt_exact(dt))
    hipLaunchKernelGGL(merge_topk_kernel<int64_t>, dim3(1), dim3(64), 0, s, count, k_in, (const int64_t*)ein, min, k,
                       (int64_t*)eout, mout);
  else
    hipLaunchKernelGGL(merge_topk_kernel<double>, dim3(1), dim3(64), 0, s, count, k_in, (const double*)ein, min, k,
                       (double*)eout, mout);
  return hipGetLastError();
}

}  // namespace qbf
