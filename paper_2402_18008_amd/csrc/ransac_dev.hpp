// Device functions for RANSAC hypothesise-and-verify: counter-based sampling
// (Philox4x32-10 + Floyd), hypothesis solve (ACA) and the inlier test.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "solver_dev.hpp"

namespace hg {

// Philox4x32-10 (Salmon et al., SC 2011): 10 rounds, key bumped by the Weyl
// constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Floyd's algorithm: 4 distinct indices of [0, n), n >= 4, in order of choice.
// Draw i maps its 32-bit word r to t = floor(r (j + 1) / 2^32) in [0, j].
__device__ __forceinline__ void floyd4(const uint32_t r[4], uint32_t n, uint32_t idx[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t j = n - 4u + static_cast<uint32_t>(i);
    const uint32_t t = __umulhi(r[i], j + 1u);
    bool taken = false;
#pragma unroll
    for (int k = 0; k < i; ++k) taken |= idx[k] == t;
    idx[i] = taken ? j : t;
  }
}

// Hypothesis `hyp` of pair `pair`: its 4 sample indices and the scaled float H.
// Points [base, base + n) of the planes x1 y1 x2 y2 (stride ld). Returns the
// solver flags (non-zero = not a valid hypothesis); n < 4 gives kZeroH.
__device__ __forceinline__ uint32_t make_hypothesis(const float *__restrict__ corr, int64_t ld,
                                                    int64_t base, uint32_t n, uint32_t k0,
                                                    uint32_t k1, uint32_t hyp, uint32_t pair,
                                                    float *h) {
  if (n < 4u) {
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = 0.0f;
    return kZeroH;
  }
  uint32_t c[4] = {hyp, pair, 0u, 0u};
  philox4x32_10(c, k0, k1);
  uint32_t idx[4];
  floyd4(c, n, idx);
  float s[8], d[8];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + idx[k];
    s[2 * k] = corr[i];
    s[2 * k + 1] = corr[ld + i];
    d[2 * k] = corr[2 * ld + i];
    d[2 * k + 1] = corr[3 * ld + i];
  }
  return solve_quad<0>(s, d, h);
}

// Division-free inlier test of one correspondence against H (float), on the
// scoring form of the hypothesis: rows 1 and 2 of H multiplied by c = 1/tau
// (score_form) and the target point multiplied by c as well (x2c = x2 c,
// y2c = y2 c). With u, v, w = H (x1, y1, 1):
//   ru = c u - x2c w, rv = c v - y2c w  (= c (u - x2 w), c (v - y2 w)),
//   inlier iff ru^2 + rv^2 <= w^2, i.e. ||pi(H x1) - x2|| <= tau for w != 0.
// Folding tau into the operands saves one instruction per (hypothesis, point)
// over comparing against (tau w)^2: 6 FMA, 2 FMA, mul + FMA, mul, compare.
__device__ __forceinline__ void score_form(const float *H, float c, float *hs) {
#pragma unroll
  for (int k = 0; k < 6; ++k) hs[k] = H[k] * c;
#pragma unroll
  for (int k = 6; k < 9; ++k) hs[k] = H[k];
}

__device__ __forceinline__ bool inlier(const float *hs, float x1, float y1, float x2c,
                                       float y2c) {
  const float u = fmaf(hs[0], x1, fmaf(hs[1], y1, hs[2]));
  const float v = fmaf(hs[3], x1, fmaf(hs[4], y1, hs[5]));
  const float w = fmaf(hs[6], x1, fmaf(hs[7], y1, hs[8]));
  const float ru = fmaf(-x2c, w, u);
  const float rv = fmaf(-y2c, w, v);
  const float d = fmaf(rv, rv, ru * ru);
  return d <= w * w;
}

// Packed argmax key: larger count wins, then the lower hypothesis index.
// 0 means "no valid hypothesis".
__device__ __forceinline__ unsigned long long pack_key(uint32_t count, uint32_t hyp) {
  return (static_cast<unsigned long long>(count + 1u) << 32) |
         static_cast<unsigned long long>(0xFFFFFFFFu - hyp);
}

}  // namespace hg
