// Streaming reference kernels. They are not part of the method: they move the
// bytes of the solver kernels without their arithmetic. A plain copy calibrates
// the hardware byte counters. A plane-to-plane stream with a solver's exact
// per-lane access pattern (same planes, same launch shape, non-temporal loads
// and stores) measures the ceiling of that read/write mix.
#include "common.hpp"

namespace hg {

constexpr int kStreamThreads = 512;   // the solver kernels' workgroup size
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Plain copy, 16 bytes per lane per step (both pointers 16-byte aligned).
__global__ __launch_bounds__(kStreamThreads) void stream_copy4_kernel(
    const f32x4 *__restrict__ src, f32x4 *__restrict__ dst, int64_t n4) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n4;
       i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Plain copy, one float per lane (tails and unaligned pointers).
__global__ __launch_bounds__(kStreamThreads) void stream_copy_kernel(const float *__restrict__ src,
                                                                    float *__restrict__ dst,
                                                                    int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// One element per lane: NI input planes in, NO output planes (and a flag byte)
// out, plane stride ld. Output plane j holds in[j mod NI] + in[j + NO] (the
// second term only where j + NO < NI), so every input is consumed and every
// output depends on the loads.
template <int NI, int NO>
__global__ __launch_bounds__(kStreamThreads) void stream_planes_kernel(
    const float *__restrict__ in, int64_t n, int64_t ld, float *__restrict__ out,
    uint8_t *__restrict__ flags) {
  static_assert(NI <= 2 * NO, "every input plane must reach an output");
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
       q += stride) {
    float v[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) v[k] = __builtin_nontemporal_load(in + k * ld + q);
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const float o = j + NO < NI ? v[j % NI] + v[j + NO] : v[j % NI];
      __builtin_nontemporal_store(o, out + j * ld + q);
    }
    if (flags) __builtin_nontemporal_store(static_cast<uint8_t>(v[0] < 0.0f), flags + q);
  }
}

static unsigned stream_grid(int64_t n) {
  const int64_t blocks = (n + kStreamThreads - 1) / kStreamThreads;
  return static_cast<unsigned>(blocks > 0x7FFFFFFF ? 0x7FFFFFFF : blocks);
}

}  // namespace hg

extern "C" int hg_stream_copy(const float *src, float *dst, int64_t n, void *stream) {
  hg::clear_error();
  HG_REQUIRE(n >= 0, "hg_stream_copy: n < 0");
  if (n == 0) return HG_OK;
  HG_REQUIRE(src && dst, "hg_stream_copy: NULL pointer");
  const hipStream_t s = hg::as_stream(stream);
  int64_t done = 0;
  if (hg::aligned(src, 16) && hg::aligned(dst, 16) && n >= 4) {
    const int64_t n4 = n / 4;
    hipLaunchKernelGGL(hg::stream_copy4_kernel, dim3(hg::stream_grid(n4)),
                       dim3(hg::kStreamThreads), 0, s, reinterpret_cast<const hg::f32x4 *>(src),
                       reinterpret_cast<hg::f32x4 *>(dst), n4);
    if (int st = hg::launched("stream_copy4_kernel")) return st;
    done = 4 * n4;
  }
  if (done == n) return HG_OK;
  hipLaunchKernelGGL(hg::stream_copy_kernel, dim3(hg::stream_grid(n - done)),
                     dim3(hg::kStreamThreads), 0, s, src + done, dst + done, n - done);
  return hg::launched("stream_copy_kernel");
}

extern "C" int hg_stream_planes(const float *in, int32_t n_in, float *out, int32_t n_out,
                                uint8_t *flags, int64_t n, int64_t ld, void *stream) {
  hg::clear_error();
  HG_REQUIRE(n >= 0, "hg_stream_planes: n < 0");
  if (n == 0) return HG_OK;
  HG_REQUIRE(in && out, "hg_stream_planes: NULL in or out");
  HG_REQUIRE(ld >= n && ld <= INT64_MAX / 16, "hg_stream_planes: ld out of range");
  const hipStream_t s = hg::as_stream(stream);
  const dim3 g(hg::stream_grid(n)), b(hg::kStreamThreads);
  if (n_in == 16 && n_out == 9)
    hipLaunchKernelGGL((hg::stream_planes_kernel<16, 9>), g, b, 0, s, in, n, ld, out, flags);
  else if (n_in == 8 && n_out == 9)
    hipLaunchKernelGGL((hg::stream_planes_kernel<8, 9>), g, b, 0, s, in, n, ld, out, flags);
  else if (n_in == 12 && n_out == 6)
    hipLaunchKernelGGL((hg::stream_planes_kernel<12, 6>), g, b, 0, s, in, n, ld, out, flags);
  else
    return hg::fail(HG_EINVAL, "hg_stream_planes: unsupported shape %d -> %d planes", n_in,
                    n_out);
  return hg::launched("stream_planes_kernel");
}
