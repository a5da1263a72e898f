// Wave-level data movement on gfx950 without LDS permutes: DPP moves of 64-bit
// values, lane reads, and a wave sum in a fixed order.
#pragma once

#include <hip/hip_runtime.h>

namespace dg {

// Wave sum with DPP row operations and lane reads (no LDS permutes); every lane of
// the wave must be active.  Within each row of 16 lanes: xor-1 and xor-2 quad
// permutes, then the half-row and row mirrors; the four row sums are then read
// from lanes 0, 16, 32, 48 and added in a fixed order (result uniform).
// (CTRL patterns whose every lane reads a valid lane of its row: no "old" value)
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_read(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x140>(v);   // row_mirror
  return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}


// sum over each group of 8 consecutive lanes (all 8 active), the same value on every
// lane of the group: two quad permutes, then the xor-4 partner through ds_bpermute
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  return v + __shfl_xor(v, 4);
}

}  // namespace dg
