// Wavefront (64-lane) primitives used by the enumeration kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qbf {

// DPP row_newbcast:Q — every lane of a 16-lane row receives lane Q of its row.
// Folded by the compiler into the consuming VOP2 (v_add_f32_dpp / v_add_u32_dpp).
template <int Q>
__device__ __forceinline__ float row_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + Q, 0xf, 0xf, false));
}
template <int Q>
__device__ __forceinline__ int32_t row_bcast(int32_t v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x150 + Q, 0xf, 0xf, false);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t readlane_u32(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
  uint32_t lo = readlane_u32((uint32_t)v, l), hi = readlane_u32((uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double readlane_f64(double v, int l) {
  return __builtin_bit_cast(double, readlane_u64(__builtin_bit_cast(uint64_t, v), l));
}
__device__ __forceinline__ int64_t readlane_i64(int64_t v, int l) {
  return (int64_t)readlane_u64((uint64_t)v, l);
}
// Make a value held identically by all lanes provably uniform (SGPR).
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double uniform_f64(double v) {
  return __builtin_bit_cast(double, uniform_u64(__builtin_bit_cast(uint64_t, v)));
}
__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }

// (ka, ma) strictly before (kb, mb) in (key, mask) order.
template <class K>
__device__ __forceinline__ bool before(K ka, uint64_t ma, K kb, uint64_t mb) {
  return ka < kb || (ka == kb && ma < mb);
}

// Sorted candidate list spread over the wave: lane q < kp holds entry q in
// ascending (key, mask) order; unused entries hold (+inf, ~0).  Inserts the
// wave-uniform candidate (ck, cm) if it ranks among the first kp entries.
// Returns true when the list changed.  Must be called with all lanes active.
__device__ __forceinline__ bool list_insert(double& lkey, uint64_t& lmask, double ck, uint64_t cm, int kp,
                                            int lane) {
  const bool pre = lane < kp && before(lkey, lmask, ck, cm);
  const int pos = __popcll(ballot(pre));
  if (pos >= kp) return false;
  const double pk = __shfl_up(lkey, 1);
  const uint64_t pm = __shfl_up(lmask, 1);
  if (lane > pos && lane < kp) {
    lkey = pk;
    lmask = pm;
  }
  if (lane == pos) {
    lkey = ck;
    lmask = cm;
  }
  return true;
}

// Ascending bitonic sort of one (key, mask) pair per lane over the 64 lanes.
template <class K>
__device__ __forceinline__ void wave_sort(K& key, uint64_t& mask, int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const K pk = __shfl_xor(key, j);
      const uint64_t pm = __shfl_xor(mask, j);
      const bool up = (lane & k) == 0;
      const bool lower = (lane & j) == 0;
      const bool keep_min = (lower == up);
      const bool take = keep_min ? before(pk, pm, key, mask) : before(key, mask, pk, pm);
      if (take) {
        key = pk;
        mask = pm;
      }
    }
  }
}

}  // namespace qbf
