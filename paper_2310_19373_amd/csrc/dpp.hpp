// Wave-wide minimum and sum of a float32 in every lane, without LDS: DPP
// moves within each row of 16 lanes (xor 1 and xor 2 by quad permutations,
// then the half-row and row mirrors), then the four rows by lane reads.
#pragma once

#include <hip/hip_runtime.h>

namespace qbf {

template <int Ctrl>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), Ctrl, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_f32(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ float wave_min_f32(float v) {
  v = fminf(v, dpp_mov<0xB1>(v));   // quad_perm [1, 0, 3, 2]
  v = fminf(v, dpp_mov<0x4E>(v));   // quad_perm [2, 3, 0, 1]
  v = fminf(v, dpp_mov<0x141>(v));  // row_half_mirror
  v = fminf(v, dpp_mov<0x140>(v));  // row_mirror
  return fminf(fminf(lane_f32(v, 0), lane_f32(v, 16)), fminf(lane_f32(v, 32), lane_f32(v, 48)));
}
__device__ __forceinline__ float wave_sum_f32(float v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  v += dpp_mov<0x140>(v);
  return (lane_f32(v, 0) + lane_f32(v, 16)) + (lane_f32(v, 32) + lane_f32(v, 48));
}

}  // namespace qbf
