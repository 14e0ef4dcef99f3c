// Cross-lane moves within one 64-lane wavefront, by DPP (data-parallel primitives) on the
// VALU instead of an LDS permute: wave_shr:1 gives lane l the value of lane l-1,
// wave_shl:1 the value of lane l+1; lanes without a source lane receive 0 (bound_ctrl), or,
// in the _or variants, keep the fill value given for them.
#pragma once
#include <hip/hip_runtime.h>

namespace mgk {

constexpr int kDppWaveShl1 = 0x130;  // lane l <- lane l+1
constexpr int kDppWaveShr1 = 0x138;  // lane l <- lane l-1

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v)
{
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
  const int lo = dpp_i32<CTRL>(__double2loint(v));
  const int hi = dpp_i32<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
  return __int_as_float(dpp_i32<CTRL>(__float_as_int(v)));
}

// value of the lane below (l-1) / above (l+1)
template <typename T>
__device__ __forceinline__ T from_lane_below(T v) { return dpp<kDppWaveShr1>(v); }
template <typename T>
__device__ __forceinline__ T from_lane_above(T v) { return dpp<kDppWaveShl1>(v); }

// The same moves where the lane without a source lane (lane 0 for wave_shr, lane 63 for
// wave_shl) receives its own value of `fill` instead of 0.
template <int CTRL>
__device__ __forceinline__ double dpp_or(double v, double fill)
{
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(fill), __double2loint(v), CTRL, 0xF,
                                             0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(fill), __double2hiint(v), CTRL, 0xF,
                                             0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_lane_below_or(double v, double fill)
{
  return dpp_or<kDppWaveShr1>(v, fill);
}
__device__ __forceinline__ double from_lane_above_or(double v, double fill)
{
  return dpp_or<kDppWaveShl1>(v, fill);
}

// The value of lane `src` (a constant) in every lane.
__device__ __forceinline__ double lane_value(double v, int src)
{
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

}  // namespace mgk
