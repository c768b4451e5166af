// Cross-lane helpers shared by the kernels that reduce doubles over a
// workgroup.
#pragma once

#include <hip/hip_runtime.h>

namespace hg {

// Sum of a double over each row of 16 lanes, in the row's last lane: an
// inclusive scan by DPP row shifts of its two 32-bit halves (lanes shifted in
// from outside the row read 0). The additions run in a fixed order, and no
// LDS round trip is involved, unlike shuffles.
__device__ __forceinline__ double row_sum16_f64(double x) {
#define HG_ROW_SHR(N)                                                              \
  {                                                                                \
    const int lo = __double2loint(x), hi = __double2hiint(x);                      \
    const int slo = __builtin_amdgcn_update_dpp(0, lo, 0x110 + N, 0xF, 0xF, false); \
    const int shi = __builtin_amdgcn_update_dpp(0, hi, 0x110 + N, 0xF, 0xF, false); \
    x += __hiloint2double(shi, slo);                                               \
  }
  HG_ROW_SHR(1)
  HG_ROW_SHR(2)
  HG_ROW_SHR(4)
  HG_ROW_SHR(8)
#undef HG_ROW_SHR
  return x;
}

}  // namespace hg
