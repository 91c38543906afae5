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

template <class E>
struct Ar;
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

// Next work unit of the persistent queue, identical in all lanes.  Every lane
// issues the atomic (increment 1 from lane 0, 0 from the others) and the
// result of the first lane is broadcast: there is no lane-divergent branch
// around the pull, so the loop exit it controls is uniform.  Must be called
// with all lanes active.
__device__ __forceinline__ uint64_t next_unit(const Views& v, int lane) {
  const uint64_t r = atomicAdd((unsigned long long*)&v.hdr->unit_counter, lane == 0 ? 1ull : 0ull);
  return uniform_u64(r);
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

// Per-lane init of a work unit.  The lane owns the prefix p (lane and tile
// bits, at positions B+no and up).  Returns E_P(p); fills the inner table
// C'(j) = E_I(j) + X_PI(p, j) (invalid lanes and inner states get the type's
// sentinel) and writes the cross fields c_l = sum_{v in prefix} S_{B+l, v} x_v
// of the outer bits to the wave's LDS table (entry l*64 + lane).
template <class E, int NB>
__device__ __forceinline__ typename Ar<E>::W lane_init(const Views& v, int b, const InstU& I, uint64_t p, bool valid,
                                                       typename Ar<E>::W* myc, int lane, E (&C)[NB]) {
  using W = typename Ar<E>::W;
  const int pos0 = I.B + I.no;
  const int64_t nm = v.nmax;
  const gptr<const W> qs = gp((const W*)v.qs) + (int64_t)b * nm * nm;
  const gptr<const W> ei = gp((const W*)v.ei) + (int64_t)b * 64;
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
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    W cj = ei[j];
#pragma unroll
    for (int u = 0; u < 6; ++u)
      if ((j >> u) & 1) cj += cI[u];
    C[j] = (valid && j < (1 << I.B)) ? (E)cj : Ar<E>::inv();
  }
  return EP;
}

}  // namespace qbf
