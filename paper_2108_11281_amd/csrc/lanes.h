// Whole-wave lane shifts (device code of the stencil kernels).
#pragma once

#include <hip/hip_runtime.h>

namespace mlmc {

// whole-wave lane shifts by one (DPP wave_shr:1 / wave_shl:1): lane i receives
// lane i-1 (shr) or lane i+1 (shl); the lane without a source keeps its value
__device__ __forceinline__ float wave_shr1(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x138,
                                                    0xf, 0xf, false));
}
__device__ __forceinline__ float wave_shl1(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x130,
                                                    0xf, 0xf, false));
}
__device__ __forceinline__ double wave_shr1(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = (int)(u & 0xffffffffll), hi = (int)(u >> 32);
  const int l2 = __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false);
  const int h2 = __builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false);
  return __longlong_as_double(((long long)h2 << 32) | (unsigned int)l2);
}
__device__ __forceinline__ double wave_shl1(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = (int)(u & 0xffffffffll), hi = (int)(u >> 32);
  const int l2 = __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false);
  const int h2 = __builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false);
  return __longlong_as_double(((long long)h2 << 32) | (unsigned int)l2);
}

}  // namespace mlmc
