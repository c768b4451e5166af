// Batched 4-point solver: one quadruple per lane (scalar path) or four
// consecutive quadruples per lane with 16-byte loads and stores from the SoA
// planes (vector path). Memory-bound: 64 B in and 36 B (+1 flag byte) out per
// quadruple; the double-precision arithmetic hides under the HBM time.
#include "common.hpp"
#include "solver_dev.hpp"

namespace hg {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int METHOD>
__global__ __launch_bounds__(256) void solve4_vec4_kernel(const float *__restrict__ src,
                                                          const float *__restrict__ dst,
                                                          int64_t nvec, int64_t ld,
                                                          float *__restrict__ H,
                                                          uint8_t *__restrict__ flags) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < nvec;
       i += stride) {
    const int64_t q = i * 4;
    f4 a[8], b[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      a[k] = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(src + k * ld + q));
      b[k] = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(dst + k * ld + q));
    }
    float h[4][9];
    uint32_t packed = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float s[8], d[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        s[k] = a[k][v];
        d[k] = b[k][v];
      }
      packed |= solve_quad<METHOD>(s, d, h[v]) << (8 * v);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const f4 o = {h[0][k], h[1][k], h[2][k], h[3][k]};
      __builtin_nontemporal_store(o, reinterpret_cast<f4 *>(H + k * ld + q));
    }
    if (flags) __builtin_nontemporal_store(packed, reinterpret_cast<uint32_t *>(flags + q));
  }
}

template <int METHOD>
__global__ __launch_bounds__(256) void solve4_scalar_kernel(const float *__restrict__ src,
                                                            const float *__restrict__ dst,
                                                            int64_t first, int64_t n, int64_t ld,
                                                            float *__restrict__ H,
                                                            uint8_t *__restrict__ flags) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t q = first + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
       q += stride) {
    float s[8], d[8], h[9];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      s[k] = src[k * ld + q];
      d[k] = dst[k * ld + q];
    }
    const uint32_t f = solve_quad<METHOD>(s, d, h);
#pragma unroll
    for (int k = 0; k < 9; ++k) H[k * ld + q] = h[k];
    if (flags) flags[q] = static_cast<uint8_t>(f);
  }
}

static unsigned grid_for(int64_t items, int threads) {
  const int64_t b = (items + threads - 1) / threads;
  const int64_t cap = 1 << 20;   // beyond this the grid-stride loop takes over
  return static_cast<unsigned>(b < 1 ? 1 : (b > cap ? cap : b));
}

template <int METHOD>
static int launch_solve(const float *src, const float *dst, int64_t n, int64_t ld, float *H,
                        uint8_t *flags, hipStream_t s) {
  const bool vec = aligned(src, 16) && aligned(dst, 16) && aligned(H, 16) &&
                   (flags == nullptr || aligned(flags, 4)) && (ld % 4 == 0);
  int64_t done = 0;
  if (vec && n >= 4) {
    const int64_t nvec = n / 4;
    hipLaunchKernelGGL(solve4_vec4_kernel<METHOD>, dim3(grid_for(nvec, 256)), dim3(256), 0, s,
                       src, dst, nvec, ld, H, flags);
    if (int st = launched("solve4_vec4_kernel")) return st;
    done = nvec * 4;
  }
  if (done < n) {
    hipLaunchKernelGGL(solve4_scalar_kernel<METHOD>, dim3(grid_for(n - done, 256)), dim3(256), 0,
                       s, src, dst, done, n, ld, H, flags);
    if (int st = launched("solve4_scalar_kernel")) return st;
  }
  return HG_OK;
}

}  // namespace hg

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
