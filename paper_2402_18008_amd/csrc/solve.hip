// Batched 4-point solver: one quadruple per lane. Each wave reads 256
// contiguous bytes from each of the 16 input planes and writes 256 bytes to
// each of the 9 output planes (plus 64 flag bytes): memory-bound at 101 B per
// quadruple, with the double-precision arithmetic hidden under the HBM time.
// Measured on MI355X, this shape (512-thread workgroups, one quadruple per
// lane, a grid that covers the batch once, non-temporal loads and stores)
// streams faster than four quadruples per lane with 16-byte accesses.
#include <cmath>

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

// Simplified SK over n images of one pattern: 8 target planes in, 9 planes of
// Hbar and the flags out (69 B per problem).
__global__ __launch_bounds__(kSolveThreads) void sk_kernel(SkPattern pat,
                                                           const float *__restrict__ dst,
                                                           int64_t n, int64_t ld,
                                                           float *__restrict__ H,
                                                           uint8_t *__restrict__ flags) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
       q += stride) {
    float d[8], h[9];
#pragma unroll
    for (int k = 0; k < 8; ++k) d[k] = __builtin_nontemporal_load(dst + k * ld + q);
    const uint32_t f = solve_sk(pat, d, h);
#pragma unroll
    for (int k = 0; k < 9; ++k) __builtin_nontemporal_store(h[k], H + k * ld + q);
    if (flags) __builtin_nontemporal_store(static_cast<uint8_t>(f), flags + q);
  }
}

// Three-point affine: 6 + 6 planes in, 6 planes of A and the flags out
// (73 B per problem).
__global__ __launch_bounds__(kSolveThreads) void affine_kernel(const float *__restrict__ src,
                                                               const float *__restrict__ dst,
                                                               int64_t n, int64_t ld,
                                                               float *__restrict__ A,
                                                               uint8_t *__restrict__ flags) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
       q += stride) {
    float s[6], d[6], a[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      s[k] = __builtin_nontemporal_load(src + k * ld + q);
      d[k] = __builtin_nontemporal_load(dst + k * ld + q);
    }
    const uint32_t f = solve_affine(s, d, a);
#pragma unroll
    for (int k = 0; k < 6; ++k) __builtin_nontemporal_store(a[k], A + k * ld + q);
    if (flags) __builtin_nontemporal_store(static_cast<uint8_t>(f), flags + q);
  }
}

static unsigned one_pass_grid(int64_t n) {
  const int64_t blocks = (n + kSolveThreads - 1) / kSolveThreads;
  return static_cast<unsigned>(blocks > 0x7FFFFFFF ? 0x7FFFFFFF : blocks);
}

// Per-pattern constants of the simplified SK, in the operation order of the
// per-image steps (double precision on the host, once per call).
static SkPattern sk_pattern(const double *o, double *frame) {
  const double ONx = (o[2] - o[0]) * 0.5, ONy = (o[3] - o[1]) * 0.5;
  const double Ox = o[0] + ONx, Oy = o[1] + ONy;
  const double f = ONx * ONx + ONy * ONy;
  double dx = o[4] - Ox, dy = o[5] - Oy;
  const double P3x = ONx * dx + ONy * dy, P3y = ONx * dy - ONy * dx;
  double r = 1.0 / P3y;
  SkPattern p;
  p.P5x = P3x * r;
  p.P5y = f * r;
  dx = o[6] - Ox;
  dy = o[7] - Oy;
  const double Q3x = ONx * dx + ONy * dy, Q3y = ONx * dy - ONy * dx;
  r = 1.0 / Q3y;
  const double Q7x = Q3x * r - p.P5x, Q7y = f * r - p.P5y;
  p.kp = 1.0 / (Q7x + Q7y);
  p.km = 1.0 / (Q7x - Q7y);
  p.flags = quad_side_thin(o) ? kNearDegenerate : 0u;
  if (frame) {  // H_S1 of eq. 3_2_4
    const double tx = -(ONx * Ox + ONy * Oy), ty = ONy * Ox - ONx * Oy;
    const double m[9] = {ONx, ONy, tx, -ONy, ONx, ty, 0.0, 0.0, f};
    for (int i = 0; i < 9; ++i) frame[i] = m[i];
  }
  return p;
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

extern "C" int hg_solve_sk(const double *obj, const float *dst, int64_t n, int64_t ld, float *H,
                           uint8_t *flags, double *frame, void *stream) {
  hg::clear_error();
  HG_REQUIRE(obj, "hg_solve_sk: NULL pattern");
  for (int k = 0; k < 8; ++k)
    HG_REQUIRE(std::isfinite(obj[k]), "hg_solve_sk: pattern coordinate %d is not finite", k);
  HG_REQUIRE(n >= 0, "hg_solve_sk: n = %lld < 0", static_cast<long long>(n));
  const hg::SkPattern pat = hg::sk_pattern(obj, frame);
  if (n == 0) return HG_OK;
  HG_REQUIRE(dst && H, "hg_solve_sk: NULL dst or H");
  HG_REQUIRE(ld >= n, "hg_solve_sk: ld = %lld < n = %lld", static_cast<long long>(ld),
             static_cast<long long>(n));
  HG_REQUIRE(ld <= (INT64_MAX / 16), "hg_solve_sk: ld too large");
  hipLaunchKernelGGL(hg::sk_kernel, dim3(hg::one_pass_grid(n)), dim3(hg::kSolveThreads), 0,
                     hg::as_stream(stream), pat, dst, n, ld, H, flags);
  return hg::launched("sk_kernel");
}

extern "C" int hg_solve3_affine(const float *src, const float *dst, int64_t n, int64_t ld,
                                float *A, uint8_t *flags, void *stream) {
  hg::clear_error();
  HG_REQUIRE(n >= 0, "hg_solve3_affine: n = %lld < 0", static_cast<long long>(n));
  if (n == 0) return HG_OK;
  HG_REQUIRE(src && dst && A, "hg_solve3_affine: NULL src, dst or A");
  HG_REQUIRE(ld >= n, "hg_solve3_affine: ld = %lld < n = %lld", static_cast<long long>(ld),
             static_cast<long long>(n));
  HG_REQUIRE(ld <= (INT64_MAX / 16), "hg_solve3_affine: ld too large");
  hipLaunchKernelGGL(hg::affine_kernel, dim3(hg::one_pass_grid(n)), dim3(hg::kSolveThreads), 0,
                     hg::as_stream(stream), src, dst, n, ld, A, flags);
  return hg::launched("affine_kernel");
}
