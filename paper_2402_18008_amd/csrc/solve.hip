// Batched 4-point solver: one quadruple per lane. Each wave reads 256
// contiguous bytes from each of the 16 input planes and writes 256 bytes to
// each of the 9 output planes (plus 64 flag bytes): memory-bound at 101 B per
// quadruple, with the double-precision arithmetic hidden under the HBM time.
// Measured on MI355X, this shape (512-thread workgroups, one quadruple per
// lane, a grid that covers the batch once, non-temporal loads and stores)
// streams faster than four quadruples per lane with 16-byte accesses.
#include "common.hpp"
#include "solver_dev.hpp"

namespace hg {

constexpr int kSolveThreads = 512;

template <int METHOD>
__global__ __launch_bounds__(kSolveThreads) void solve4_kernel(const float *__restrict__ src,
                                                               const float *__restrict__ dst,
                                                               int64_t n, int64_t ld,
                                                               float *__restrict__ H,
                                                               uint8_t *__restrict__ flags) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
       q += stride) {
    float s[8], d[8], h[9];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      s[k] = __builtin_nontemporal_load(src + k * ld + q);
      d[k] = __builtin_nontemporal_load(dst + k * ld + q);
    }
    const uint32_t f = solve_quad<METHOD>(s, d, h);
#pragma unroll
    for (int k = 0; k < 9; ++k) __builtin_nontemporal_store(h[k], H + k * ld + q);
    if (flags) __builtin_nontemporal_store(static_cast<uint8_t>(f), flags + q);
  }
}

template <int METHOD>
static int launch_solve(const float *src, const float *dst, int64_t n, int64_t ld, float *H,
                        uint8_t *flags, hipStream_t s) {
  // one pass over the batch; beyond 2^31 - 1 workgroups the grid-stride loop takes over
  const int64_t blocks = (n + kSolveThreads - 1) / kSolveThreads;
  const unsigned grid = static_cast<unsigned>(blocks > 0x7FFFFFFF ? 0x7FFFFFFF : blocks);
  hipLaunchKernelGGL(solve4_kernel<METHOD>, dim3(grid), dim3(kSolveThreads), 0, s, src, dst, n,
                     ld, H, flags);
  return launched("solve4_kernel");
}

// Plain copy with the solver's access pattern (one float per lane, 512-thread
// workgroups, non-temporal): the reference for calibrating hardware byte
// counters and the streaming ceiling of that pattern.
__global__ __launch_bounds__(kSolveThreads) void stream_copy_kernel(const float *__restrict__ src,
                                                                    float *__restrict__ dst,
                                                                    int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace hg

extern "C" int hg_stream_copy(const float *src, float *dst, int64_t n, void *stream) {
  hg::clear_error();
  HG_REQUIRE(n >= 0, "hg_stream_copy: n < 0");
  if (n == 0) return HG_OK;
  HG_REQUIRE(src && dst, "hg_stream_copy: NULL pointer");
  const int64_t blocks = (n + hg::kSolveThreads - 1) / hg::kSolveThreads;
  const unsigned grid = static_cast<unsigned>(blocks > 0x7FFFFFFF ? 0x7FFFFFFF : blocks);
  hipLaunchKernelGGL(hg::stream_copy_kernel, dim3(grid), dim3(hg::kSolveThreads), 0,
                     hg::as_stream(stream), src, dst, n);
  return hg::launched("stream_copy_kernel");
}

extern "C" int hg_solve4(int method, const float *src, const float *dst, int64_t n, int64_t ld,
                         float *H, uint8_t *flags, void *stream) {
  hg::clear_error();
  HG_REQUIRE(method == HG_ACA || method == HG_SKS, "hg_solve4: unknown method %d", method);
  HG_REQUIRE(n >= 0, "hg_solve4: n = %lld < 0", static_cast<long long>(n));
  if (n == 0) return HG_OK;
  HG_REQUIRE(src && dst && H, "hg_solve4: NULL src, dst or H");
  HG_REQUIRE(ld >= n, "hg_solve4: ld = %lld < n = %lld", static_cast<long long>(ld),
             static_cast<long long>(n));
  HG_REQUIRE(ld <= (INT64_MAX / 16), "hg_solve4: ld too large");
  const hipStream_t s = hg::as_stream(stream);
  return method == HG_ACA ? hg::launch_solve<0>(src, dst, n, ld, H, flags, s)
                          : hg::launch_solve<1>(src, dst, n, ld, H, flags, s);
}
