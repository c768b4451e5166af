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

// Inlier test of one correspondence (x1, y1) -> (x2, y2) against a float H:
// the point is an inlier iff its one-way transfer error is at most tau, i.e.
// with (U, V, W) = H (x1, y1, 1) and W != 0,
//   e = (U - x2 W)^2 + (V - y2 W)^2 - (tau W)^2 <= 0.
// The kernels decide it in float32 wherever a bound on the float32 rounding
// error proves the sign of e, and in float64 otherwise, so that every
// decision is that of the float64 test below (which differs from the exact
// one only for points within ~1e-12 px of the threshold).
//
// The float32 form uses the scoring form of the hypothesis: rows 1 and 2 of H
// multiplied by c = 1/tau (score_form) and the target point multiplied by c as
// well (x2c = x2 c, y2c = y2 c). With u, v, w = hs (x1, y1, 1):
//   ru = u - x2c w, rv = v - y2c w, e32 = ru^2 + rv^2 - w^2 (= e / tau^2).
// Folding tau into the operands saves one instruction per (hypothesis, point)
// over comparing against (tau w)^2: 6 FMA, 2 FMA, mul + FMA, FMA, compare.
__device__ __forceinline__ void score_form(const float *H, float c, float *hs) {
#pragma unroll
  for (int k = 0; k < 6; ++k) hs[k] = H[k] * c;
#pragma unroll
  for (int k = 6; k < 9; ++k) hs[k] = H[k];
}

// e32 of the float32 form (inlier iff e32 <= 0 when its sign is certified);
// w receives the computed w.
__device__ __forceinline__ float test_f32(const float *hs, float x1, float y1, float x2c,
                                          float y2c, float &w) {
  const float u = fmaf(hs[0], x1, fmaf(hs[1], y1, hs[2]));
  const float v = fmaf(hs[3], x1, fmaf(hs[4], y1, hs[5]));
  w = fmaf(hs[6], x1, fmaf(hs[7], y1, hs[8]));
  const float ru = fmaf(-x2c, w, u);
  const float rv = fmaf(-y2c, w, v);
  const float d = fmaf(rv, rv, ru * ru);
  return fmaf(-w, w, d);
}

// Error bound of test_f32 over a set of points with |x1| <= mx1, |y1| <= my1,
// |x2c| <= mx2, |y2c| <= my2. With u32 = 2^-24, SU = |hs0| mx1 + |hs1| my1 +
// |hs2| (SV, SW likewise for rows 2 and 3) and
//   S = 4.1 u32 (SU + SV + (mx2 + my2) SW),
// each of ru, rv errs by at most 4.1 u32 (its row's magnitude sum + |x2c| SW)
// + u32 |ru| (the operand scalings by c, the two FMA roundings of u and w,
// the residual's rounding), w by 2.01 u32 SW, and the squares, sum and
// difference add relative roundings. For a point whose computed e32 is within
// its error E of zero, d = e32 + w^2 stays near w^2, which bounds |ru|, |rv|
// through sqrt(d); solving the resulting inequality for E gives
//   E <= (|w| k1 + k0) / 2,  k1 = 23 u32 SW + 5.5 S,  k0 = 14 S^2 + 11 u32^2 SW^2.
// So |e32| > |w| k1 + k0 proves sign(e32) = sign(e), and (the factor 2) also
// places the point outside the float64 test's much smaller error band, so
// that the float64 decision agrees. Magnitudes large enough for float32
// squares to overflow give k0 = inf (every point goes to float64).
__device__ __forceinline__ void error_bound(const float *hs, float mx1, float my1, float mx2,
                                            float my2, float &k1, float &k0) {
  constexpr float u = 5.9604645e-08f;   // 2^-24
  const float su = fmaf(fabsf(hs[0]), mx1, fmaf(fabsf(hs[1]), my1, fabsf(hs[2])));
  const float sv = fmaf(fabsf(hs[3]), mx1, fmaf(fabsf(hs[4]), my1, fabsf(hs[5])));
  const float sw = fmaf(fabsf(hs[6]), mx1, fmaf(fabsf(hs[7]), my1, fabsf(hs[8])));
  const float mag = fmaf(mx2 + my2, sw, su + sv);
  const float S = (4.1f * u) * mag;
  k1 = fmaf(23.0f * u, sw, 5.5f * S);
  const float usw = u * sw;
  // + 1e-35: absolute rounding of results in the subnormal range
  k0 = fmaf(14.0f * S, S, fmaf(11.0f * usw, usw, 1.0e-35f));
  if (!(mag + sw < 1.0e18f)) k0 = __builtin_inff();
}

// The float64 test on the original operands (float H as scored, here given
// as doubles; float coordinates and tau): the products of float operands are
// exact in the FMAs, so e is within a few double roundings of its exact
// value. W = 0 (the point maps to infinity) is an outlier.
__device__ __forceinline__ bool inlier_f64(const double *H, float x1, float y1, float x2,
                                           float y2, float tau) {
  const double X = x1, Y = y1;
  const double U = fma(H[0], X, fma(H[1], Y, H[2]));
  const double V = fma(H[3], X, fma(H[4], Y, H[5]));
  const double W = fma(H[6], X, fma(H[7], Y, H[8]));
  const double ru = fma(-static_cast<double>(x2), W, U);
  const double rv = fma(-static_cast<double>(y2), W, V);
  const double tw = static_cast<double>(tau) * W;
  return W != 0.0 && fma(-tw, tw, fma(rv, rv, ru * ru)) <= 0.0;
}

// Packed argmax key: larger count wins, then the lower hypothesis index.
// 0 means "no valid hypothesis".
__device__ __forceinline__ unsigned long long pack_key(uint32_t count, uint32_t hyp) {
  return (static_cast<unsigned long long>(count + 1u) << 32) |
         static_cast<unsigned long long>(0xFFFFFFFFu - hyp);
}

}  // namespace hg
