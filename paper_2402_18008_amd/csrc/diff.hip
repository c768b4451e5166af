// Differentiable 4-point-offset pipeline: offsets -> H (Algorithm 1, the
// tensorised ACA for a rectangle) -> bilinear inverse warp -> L1 loss, with
// hand-written backward kernels that recompute per-pixel state from H.
//
// H is carried in double precision between the stages, and every per-pixel
// step (sample position, bilinear weights, residual, gradient terms) runs in
// double on the float images: a float sample position (error ~1e-5 px) would
// move pixels across the kinks of the bilinear and L1 terms and change the
// gradient by ~1e-3 relative. One 256-thread workgroup per patch; per-patch
// sums are accumulated per thread and across the workgroup in double.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "lanes.hpp"
#include "solver_dev.hpp"

namespace hg {

constexpr int kDiffThreads = 256;

// Target corners from the offsets (TL, TR, BR, BL) of the rectangle with
// upper-left (x0, y0), width w and aspect ratio r, as ACA points M N P Q.
struct RectCorners {
  double M2x, M2y, N2x, N2y, P2x, P2y, Q2x, Q2y;
};

__device__ __forceinline__ RectCorners rect_targets(const float *o, double x0, double y0, double w,
                                                    double r) {
  const double hgt = w / r;
  RectCorners c;
  c.M2x = x0 + static_cast<double>(o[0]);
  c.M2y = y0 + static_cast<double>(o[1]);
  c.N2x = x0 + w + static_cast<double>(o[2]);
  c.N2y = y0 + static_cast<double>(o[3]);
  c.Q2x = x0 + w + static_cast<double>(o[4]);
  c.Q2y = y0 + hgt + static_cast<double>(o[5]);
  c.P2x = x0 + static_cast<double>(o[6]);
  c.P2y = y0 + hgt + static_cast<double>(o[7]);
  return c;
}

// Algorithm 1: H = [h1 h2 h3] (columns) from the target corners.
__device__ __forceinline__ void rect_aca(const RectCorners &k, double x0, double y0, double w,
                                         double r, double H[9]) {
  const double d1[3] = {k.N2x - k.M2x, k.P2x - k.M2x, k.Q2x - k.M2x};
  const double d2[3] = {k.N2y - k.M2y, k.P2y - k.M2y, k.Q2y - k.M2y};
  const double c0 = d1[1] * d2[2] - d1[2] * d2[1];
  const double c1 = d1[2] * d2[0] - d1[0] * d2[2];
  const double c2 = d1[0] * d2[1] - d1[1] * d2[0];
  const double S = c0 + c1 + c2;
  const double b[3] = {S * k.M2x, S * k.M2y, S};
  const double h1[3] = {c0 * k.N2x - b[0], c0 * k.N2y - b[1], c0 - b[2]};
  const double h2[3] = {r * (c1 * k.P2x - b[0]), r * (c1 * k.P2y - b[1]), r * (c1 - b[2])};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    H[3 * i + 0] = h1[i];
    H[3 * i + 1] = h2[i];
    H[3 * i + 2] = w * b[i] - x0 * h1[i] - y0 * h2[i];
  }
}

__global__ void rect_fwd_kernel(const float *__restrict__ off, int B, double x0, double y0,
                                double w, double r, double *__restrict__ H) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const RectCorners k = rect_targets(off + 8 * b, x0, y0, w, r);
  double h[9];
  rect_aca(k, x0, y0, w, r, h);
#pragma unroll
  for (int i = 0; i < 9; ++i) H[9 * b + i] = h[i];
}

// Reverse mode through Algorithm 1 (each step's adjoint in reverse order) for
// one patch: offsets o (8), dL/dH gHb (9) -> dL/d offsets (8, order TL TR BR BL).
__device__ __forceinline__ void rect_bwd_one(const float *o, const double *gHb, double x0,
                                             double y0, double w, double r, double *gout) {
  const RectCorners k = rect_targets(o, x0, y0, w, r);
  const double d1[3] = {k.N2x - k.M2x, k.P2x - k.M2x, k.Q2x - k.M2x};
  const double d2[3] = {k.N2y - k.M2y, k.P2y - k.M2y, k.Q2y - k.M2y};
  const double c0 = d1[1] * d2[2] - d1[2] * d2[1];
  const double c1 = d1[2] * d2[0] - d1[0] * d2[2];
  const double c2 = d1[0] * d2[1] - d1[1] * d2[0];
  const double S = c0 + c1 + c2;
  double g1[3], g2[3], g3[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    g1[i] = gHb[3 * i + 0];
    g2[i] = gHb[3 * i + 1];
    g3[i] = gHb[3 * i + 2];
  }
  double gb[3], gM2x = 0, gM2y = 0, gN2x = 0, gN2y = 0, gP2x = 0, gP2y = 0, gQ2x = 0, gQ2y = 0;
  // h3 = w b - x0 h1 - y0 h2
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gb[i] = w * g3[i];
    g1[i] -= x0 * g3[i];
    g2[i] -= y0 * g3[i];
  }
  // h2 = r (c1 p2 - b), p2 = (P2x, P2y, 1)
  double e[3] = {r * g2[0], r * g2[1], r * g2[2]};
  double gc1 = e[0] * k.P2x + e[1] * k.P2y + e[2];
  gP2x += e[0] * c1;
  gP2y += e[1] * c1;
  // h1 = c0 n2 - b, n2 = (N2x, N2y, 1)
  double gc0 = g1[0] * k.N2x + g1[1] * k.N2y + g1[2];
  gN2x += g1[0] * c0;
  gN2y += g1[1] * c0;
#pragma unroll
  for (int i = 0; i < 3; ++i) gb[i] -= e[i] + g1[i];
  // b = S m2, m2 = (M2x, M2y, 1)
  const double gS = gb[0] * k.M2x + gb[1] * k.M2y + gb[2];
  gM2x += gb[0] * S;
  gM2y += gb[1] * S;
  gc0 += gS;
  gc1 += gS;
  const double gc2 = gS;
  // c = d1 x d2
  double gd1[3] = {0, 0, 0}, gd2[3] = {0, 0, 0};
  gd1[1] += gc0 * d2[2];
  gd2[2] += gc0 * d1[1];
  gd1[2] -= gc0 * d2[1];
  gd2[1] -= gc0 * d1[2];
  gd1[2] += gc1 * d2[0];
  gd2[0] += gc1 * d1[2];
  gd1[0] -= gc1 * d2[2];
  gd2[2] -= gc1 * d1[0];
  gd1[0] += gc2 * d2[1];
  gd2[1] += gc2 * d1[0];
  gd1[1] -= gc2 * d2[0];
  gd2[0] -= gc2 * d1[1];
  // d1 = (N2x, P2x, Q2x) - M2x, d2 likewise in y
  gN2x += gd1[0];
  gP2x += gd1[1];
  gQ2x += gd1[2];
  gM2x -= gd1[0] + gd1[1] + gd1[2];
  gN2y += gd2[0];
  gP2y += gd2[1];
  gQ2y += gd2[2];
  gM2y -= gd2[0] + gd2[1] + gd2[2];
  // TL TR BR BL = M N Q P
  gout[0] = gM2x;
  gout[1] = gM2y;
  gout[2] = gN2x;
  gout[3] = gN2y;
  gout[4] = gQ2x;
  gout[5] = gQ2y;
  gout[6] = gP2x;
  gout[7] = gP2y;
}

__global__ void rect_bwd_kernel(const float *__restrict__ off, const double *__restrict__ gH, int B,
                                double x0, double y0, double w, double r,
                                float *__restrict__ goff) {
  const int bi = blockIdx.x * blockDim.x + threadIdx.x;
  if (bi >= B) return;
  double g[8];
  rect_bwd_one(off + 8 * bi, gH + 9 * bi, x0, y0, w, r, g);
#pragma unroll
  for (int i = 0; i < 8; ++i) goff[8 * bi + i] = static_cast<float>(g[i]);
}

// adj(H) (cyclic cofactor form) scaled by 2^-e so that max|G| is in [0.5, 1);
// returns e (0 if G is zero or not finite, then G = 0).
__device__ __forceinline__ int adjugate_scaled(const double *Hd, double G[9]) {
  double H[3][3];
#pragma unroll
  for (int i = 0; i < 9; ++i) H[i / 3][i % 3] = Hd[i];
  double m = 0.0;
  bool bad = false;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int a = (j + 1) % 3, b2 = (j + 2) % 3, c = (i + 1) % 3, d = (i + 2) % 3;
      const double g = H[a][c] * H[b2][d] - H[a][d] * H[b2][c];
      G[3 * i + j] = g;
      bad |= !(fabs(g) <= 1.7976931348623157e308);
      m = fmax(m, fabs(g));
    }
  if (bad || m == 0.0) {
#pragma unroll
    for (int i = 0; i < 9; ++i) G[i] = 0.0;
    return 0;
  }
  int e;
  (void)frexp(m, &e);
#pragma unroll
  for (int i = 0; i < 9; ++i) G[i] = ldexp(G[i], -e);
  return e;
}

// Bilinear sampling with zero padding, split into an address stage and an
// evaluation stage, so that a thread can issue the loads of several pixels
// before using any of them. The patch image is read as a raw buffer of its
// h w floats, whose loads return 0 at byte offsets past its end (the hardware's
// range check): a row above the image gets an offset past the end, a row below
// it lies past the end already, and the two tap columns are clamped into the
// image and masked. Offsets are 32-bit and never negative.
constexpr uint32_t kFarOffset = 0x80000000u;   // past every patch (h w <= 2^29 floats)

struct TapAddr {
  uint32_t o00, o01, o10, o11;   // byte offsets of taps (x0, y0), (x1, y0), (x0, y1), (x1, y1)
  bool x0in, x1in;               // tap columns inside the image
  double ax, ay;                 // fractional position in the cell
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t patch_buffer(const float *I, int P) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(I), 0, P * 4, 0x00020000);
}

__device__ __forceinline__ TapAddr tap_addr(double sx, double sy, int h, int w) {
  if (!(fabs(sx) < 1.0e6) || !(fabs(sy) < 1.0e6)) {   // far outside or nan: all taps outside
    sx = -4.0;
    sy = -4.0;
  }
  const double fx = floor(sx), fy = floor(sy);
  TapAddr t;
  t.ax = sx - fx;
  t.ay = sy - fy;
  const int ix = static_cast<int>(fx), iy = static_cast<int>(fy);
  // cells with a tap inside the image; any other cell has all four taps outside
  const bool near = ix >= -1 && ix < w && iy >= -1 && iy < h;
  const uint32_t row0 = near && iy >= 0 ? static_cast<uint32_t>(iy * w) * 4u : kFarOffset;
  const uint32_t row1 = near ? static_cast<uint32_t>((iy + 1) * w) * 4u : kFarOffset;
  const uint32_t c0 = static_cast<uint32_t>(max(ix, 0)) * 4u;
  const uint32_t c1 = static_cast<uint32_t>(min(ix + 1, w - 1)) * 4u;
  t.o00 = row0 + c0;
  t.o01 = row0 + c1;
  t.o10 = row1 + c0;
  t.o11 = row1 + c1;
  t.x0in = ix >= 0;
  t.x1in = ix + 1 < w;
  return t;
}

// The four taps of a cell (column-masked; rows outside read 0).
__device__ __forceinline__ void tap_load(__amdgpu_buffer_rsrc_t r, const TapAddr &t, float L[4]) {
  const float v00 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, t.o00, 0, 0));
  const float v01 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, t.o01, 0, 0));
  const float v10 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, t.o10, 0, 0));
  const float v11 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, t.o11, 0, 0));
  L[0] = t.x0in ? v00 : 0.0f;
  L[1] = t.x1in ? v01 : 0.0f;
  L[2] = t.x0in ? v10 : 0.0f;
  L[3] = t.x1in ? v11 : 0.0f;
}

struct Tap {
  double v, dvdx, dvdy;
};

template <bool GRAD>
__device__ __forceinline__ Tap tap_eval(const TapAddr &a, float L00, float L01, float L10,
                                        float L11) {
  const double I00 = static_cast<double>(L00), I01 = static_cast<double>(L01);
  const double I10 = static_cast<double>(L10), I11 = static_cast<double>(L11);
  const double top = fma(a.ax, I01 - I00, I00);
  const double bot = fma(a.ax, I11 - I10, I10);
  Tap t;
  t.v = fma(a.ay, bot - top, top);
  t.dvdx = 0.0;
  t.dvdy = 0.0;
  if (GRAD) {
    t.dvdx = fma(a.ay, (I11 - I10) - (I01 - I00), I01 - I00);
    t.dvdy = bot - top;
  }
  return t;
}

// Pixels per thread per loop iteration (loads of all of them in flight at once).
constexpr int kUnroll = 4;

// Per-thread pixel walker (NT threads): pixel i = threadIdx.x + u * NT + k *
// NT * kUnroll, with (x, y) advanced incrementally.
template <int NT>
struct PixelWalk {
  int x[kUnroll], y[kUnroll];
  int step_x, step_y, w;
  __device__ __forceinline__ PixelWalk(int w_) : w(w_) {
    constexpr int kStep = NT * kUnroll;
    step_y = kStep / w;
    step_x = kStep % w;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int i = static_cast<int>(threadIdx.x) + u * NT;
      y[u] = i / w;
      x[u] = i % w;
    }
  }
  __device__ __forceinline__ void advance() {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      x[u] += step_x;
      y[u] += step_y;
      if (x[u] >= w) {
        x[u] -= w;
        ++y[u];
      }
    }
  }
};

// Workgroup (NT threads) sum of NV per-thread partials, in double. Result valid in
// thread 0. Each row of 16 lanes sums its values (row_sum16_f64), then thread k
// adds the rows' partials of value k in row order: a fixed order, so the result
// is deterministic.
template <int NV, int NT>
__device__ __forceinline__ void block_sum(const double (&v)[NV], double (&out)[NV]) {
  constexpr int kRows = NT / 16;
  static_assert(NV <= NT, "one thread per value");
  __shared__ double red[NV][kRows];
  __shared__ double tot[NV];
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double r = row_sum16_f64(v[k]);
    if ((t & 15) == 15) red[k][t >> 4] = r;
  }
  __syncthreads();
  if (t < NV) {
    double x = red[t][0];
    for (int q = 1; q < kRows; ++q) x += red[t][q];
    tot[t] = x;
  }
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = tot[k];
  }
}

// Per-patch G = 2^-e adj(H) shared by the workgroup, read back into scalar
// registers (it is uniform): 18 fewer vector registers per lane, which lets
// the backward kernels run 4 waves per SIMD (one 256-thread patch per SIMD
// slot, all patches of a 1024-patch batch resident at once on 256 CUs).
__device__ __forceinline__ void load_G(const double *H, double G[9], int &e) {
  __shared__ double Gs[9];
  __shared__ int es;
  if (threadIdx.x == 0) {
    double g[9];
    es = adjugate_scaled(H, g);
#pragma unroll
    for (int i = 0; i < 9; ++i) Gs[i] = g[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const uint64_t v = static_cast<uint64_t>(__double_as_longlong(Gs[i]));
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    G[i] = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
  }
  e = __builtin_amdgcn_readfirstlane(es);
}

// 1/q in double: a single-precision reciprocal estimate refined by two
// Newton steps (relative error ~2^-52, no special-case handling needed since
// G is power-of-two normalised; q outside the float range gives a non-finite
// position, which samples as outside the image).
__device__ __forceinline__ double recip(double q) {
  double r = static_cast<double>(__builtin_amdgcn_rcpf(static_cast<float>(q)));
  r = fma(fma(-q, r, 1.0), r, r);
  r = fma(fma(-q, r, 1.0), r, r);
  return r;
}

__device__ __forceinline__ void sample_pos(const double *G, double x, double y, double &sx,
                                           double &sy, double &iq2) {
  const double q0 = fma(G[0], x, fma(G[1], y, G[2]));
  const double q1 = fma(G[3], x, fma(G[4], y, G[5]));
  const double q2 = fma(G[6], x, fma(G[7], y, G[8]));
  iq2 = recip(q2);
  sx = q0 * iq2;
  sy = q1 * iq2;
}

// One patch b per workgroup; Hb: its 9 entries of H (global or LDS).
// MODE 0: loss only; 2: stored warp only (rounded to float).
template <int MODE, int NT>
__device__ __forceinline__ void warp_fwd_block(const double *Hb, const float *__restrict__ img,
                                               const float *__restrict__ tgt, int h, int w, int b,
                                               float *__restrict__ loss,
                                               float *__restrict__ warped) {
  double G[9];
  int e;
  load_G(Hb, G, e);
  const int P = h * w;
  const __amdgpu_buffer_rsrc_t rs = patch_buffer(img + static_cast<int64_t>(b) * P, P);
  // the target as a buffer too: indices past the patch (the last loop's tail) read 0
  const __amdgpu_buffer_rsrc_t rt = patch_buffer(MODE == 0 ? tgt + static_cast<int64_t>(b) * P
                                                           : img, P);
  double acc[1] = {0.0};
  PixelWalk<NT> pw(w);
  for (int i0 = threadIdx.x; i0 < P; i0 += NT * kUnroll) {
    TapAddr ta[kUnroll];
    float L[kUnroll][4], tv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      double sx, sy, iq2;
      sample_pos(G, static_cast<double>(pw.x[u]), static_cast<double>(pw.y[u]), sx, sy, iq2);
      ta[u] = tap_addr(sx, sy, h, w);
      tap_load(rs, ta[u], L[u]);
      if (MODE == 0)
        tv[u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
            rt, static_cast<uint32_t>(i0 + u * NT) * 4u, 0, 0));
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int i = i0 + u * NT;
      if (i < P) {
        const double v = tap_eval<false>(ta[u], L[u][0], L[u][1], L[u][2], L[u][3]).v;
        if (MODE == 2) warped[static_cast<int64_t>(b) * P + i] = static_cast<float>(v);
        if (MODE == 0) acc[0] += fabs(v - static_cast<double>(tv[u]));
      }
    }
    pw.advance();
  }
  if (MODE == 0) {
    double s[1];
    block_sum<1, NT>(acc, s);
    if (threadIdx.x == 0) loss[b] = static_cast<float>(s[0] / static_cast<double>(P));
  }
}

template <int MODE, int NT>
__global__ __launch_bounds__(NT) void warp_fwd_kernel(const double *__restrict__ H,
                                                                const float *__restrict__ img,
                                                                const float *__restrict__ tgt,
                                                                int h, int w,
                                                                float *__restrict__ loss,
                                                                float *__restrict__ warped) {
  warp_fwd_block<MODE, NT>(H + 9 * blockIdx.x, img, tgt, h, w, blockIdx.x, loss, warped);
}

// dL/dH from dL/dG (G = 2^-e adj(H)), thread 0, double precision.
__device__ __forceinline__ void adjugate_backward(const double *Hd, const double gG[9], int e,
                                                  double *gHout) {
  double H[3][3], gH[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int i = 0; i < 9; ++i) H[i / 3][i % 3] = Hd[i];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double g = ldexp(gG[3 * i + j], -e);
      const int a = (j + 1) % 3, b2 = (j + 2) % 3, c = (i + 1) % 3, d = (i + 2) % 3;
      gH[a][c] += g * H[b2][d];
      gH[b2][d] += g * H[a][c];
      gH[a][d] -= g * H[b2][c];
      gH[b2][c] -= g * H[a][d];
    }
#pragma unroll
  for (int i = 0; i < 9; ++i) gHout[i] = gH[i / 3][i % 3];
}

// One patch b per workgroup; Hb: its 9 entries of H (global or LDS); thread 0
// writes dL/dH to gHout (9 doubles).
// FROM_STORED = false: recompute r = I_w - T and use sign(r) gl, gl = grad_loss / (h w);
// FROM_STORED = true: read dL/dI_w from grad_warped.
template <bool FROM_STORED, int NT>
__device__ __forceinline__ void warp_bwd_block(const double *Hb, const float *__restrict__ img,
                                               const float *__restrict__ tgt, double gl,
                                               const float *__restrict__ grad_warped, int h,
                                               int w, int b, double *gHout) {
  double G[9];
  int e;
  load_G(Hb, G, e);
  const int P = h * w;
  const __amdgpu_buffer_rsrc_t rs = patch_buffer(img + static_cast<int64_t>(b) * P, P);
  const float *T = FROM_STORED ? grad_warped + static_cast<int64_t>(b) * P
                               : tgt + static_cast<int64_t>(b) * P;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  PixelWalk<NT> pw(w);
  for (int i0 = threadIdx.x; i0 < P; i0 += NT * kUnroll) {
    TapAddr ta[kUnroll];
    double sx[kUnroll], sy[kUnroll], iq2[kUnroll];
    float L[kUnroll][4], tv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      sample_pos(G, static_cast<double>(pw.x[u]), static_cast<double>(pw.y[u]), sx[u], sy[u],
                 iq2[u]);
      ta[u] = tap_addr(sx[u], sy[u], h, w);
      tap_load(rs, ta[u], L[u]);
      tv[u] = T[min(i0 + u * NT, P - 1)];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (i0 + u * NT >= P) continue;
      const Tap t = tap_eval<true>(ta[u], L[u][0], L[u][1], L[u][2], L[u][3]);
      double g;
      if (FROM_STORED) {
        g = static_cast<double>(tv[u]);
      } else {
        const double r = t.v - static_cast<double>(tv[u]);
        g = (r > 0.0) ? gl : ((r < 0.0) ? -gl : 0.0);
      }
      const double xf = static_cast<double>(pw.x[u]), yf = static_cast<double>(pw.y[u]);
      const double gx = g * t.dvdx, gy = g * t.dvdy;
      const double a0 = gx * iq2[u], a1 = gy * iq2[u];
      const double a2 = -(gx * sx[u] + gy * sy[u]) * iq2[u];
      acc[0] = fma(a0, xf, acc[0]);
      acc[1] = fma(a0, yf, acc[1]);
      acc[2] += a0;
      acc[3] = fma(a1, xf, acc[3]);
      acc[4] = fma(a1, yf, acc[4]);
      acc[5] += a1;
      acc[6] = fma(a2, xf, acc[6]);
      acc[7] = fma(a2, yf, acc[7]);
      acc[8] += a2;
    }
    pw.advance();
  }
  double gG[9];
  block_sum<9, NT>(acc, gG);
  if (threadIdx.x == 0) adjugate_backward(Hb, gG, e, gHout);
}

template <bool FROM_STORED, int NT>
__global__ __launch_bounds__(NT) void warp_bwd_kernel(
    const double *__restrict__ H, const float *__restrict__ img, const float *__restrict__ tgt,
    const float *__restrict__ grad_loss, const float *__restrict__ grad_warped, int h, int w,
    double *__restrict__ grad_H) {
  const int b = blockIdx.x;
  const double gl =
      FROM_STORED ? 0.0 : static_cast<double>(grad_loss[b]) / static_cast<double>(h * w);
  warp_bwd_block<FROM_STORED, NT>(H + 9 * b, img, tgt, gl, grad_warped, h, w, b, grad_H + 9 * b);
}

// ---- fused offsets -> loss and offsets -> gradient (one workgroup per patch) --
// Algorithm 1 runs in thread 0 of the patch's workgroup into LDS, then the
// warp; the backward also runs Algorithm 1's reverse mode in thread 0. The
// arithmetic is that of the separate kernels, in the same order.
struct RectArgs {
  double x0, y0, w, r;
};

__device__ __forceinline__ void rect_to_lds(const float *o, const RectArgs &ra, double *Hs) {
  if (threadIdx.x == 0) {
    double hh[9];
    rect_aca(rect_targets(o, ra.x0, ra.y0, ra.w, ra.r), ra.x0, ra.y0, ra.w, ra.r, hh);
#pragma unroll
    for (int i = 0; i < 9; ++i) Hs[i] = hh[i];
  }
  __syncthreads();
}

template <int NT>
__global__ __launch_bounds__(NT) void photo_fwd_kernel(const float *__restrict__ off,
                                                                 const float *__restrict__ img,
                                                                 const float *__restrict__ tgt,
                                                                 int h, int w, RectArgs ra,
                                                                 float *__restrict__ loss) {
  __shared__ double Hs[9];
  rect_to_lds(off + 8 * blockIdx.x, ra, Hs);
  warp_fwd_block<0, NT>(Hs, img, tgt, h, w, blockIdx.x, loss, nullptr);
}

// grad_offsets = grad_loss[b] dL_b/d offsets_b; with STEP, instead
// offsets_b -= step * float(dL_b/d offsets_b) in place (grad_loss = 1).
template <bool STEP, int NT>
__global__ __launch_bounds__(NT) void photo_bwd_kernel(
    float *__restrict__ off, const float *__restrict__ img, const float *__restrict__ tgt,
    const float *__restrict__ grad_loss, int h, int w, RectArgs ra, float step,
    float *__restrict__ goff) {
  __shared__ double Hs[9];
  __shared__ double gHs[9];
  const int b = blockIdx.x;
  rect_to_lds(off + 8 * b, ra, Hs);
  const double gl = static_cast<double>(STEP ? 1.0f : grad_loss[b]) / static_cast<double>(h * w);
  warp_bwd_block<false, NT>(Hs, img, tgt, gl, nullptr, h, w, b, gHs);
  if (threadIdx.x == 0) {
    double g[8];
    rect_bwd_one(off + 8 * b, gHs, ra.x0, ra.y0, ra.w, ra.r, g);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float gf = static_cast<float>(g[i]);
      if (STEP)
        off[8 * b + i] = off[8 * b + i] - step * gf;
      else
        goff[8 * b + i] = gf;
    }
  }
}

__global__ void l1_fwd_kernel(const float *__restrict__ warped, const float *__restrict__ tgt,
                              int64_t P, float *__restrict__ loss) {
  const int b = blockIdx.x;
  double acc[1] = {0.0};
#pragma unroll 4
  for (int64_t i = threadIdx.x; i < P; i += kDiffThreads)
    acc[0] += fabs(static_cast<double>(warped[b * P + i]) - static_cast<double>(tgt[b * P + i]));
  double s[1];
  block_sum<1, kDiffThreads>(acc, s);
  if (threadIdx.x == 0) loss[b] = static_cast<float>(s[0] / static_cast<double>(P));
}

__global__ void l1_bwd_kernel(const float *__restrict__ warped, const float *__restrict__ tgt,
                              const float *__restrict__ grad_loss, int64_t P,
                              float *__restrict__ gw) {
  const int b = blockIdx.x;
  const float gl = static_cast<float>(static_cast<double>(grad_loss[b]) / static_cast<double>(P));
#pragma unroll 4
  for (int64_t i = threadIdx.x; i < P; i += kDiffThreads) {
    const float r = warped[b * P + i] - tgt[b * P + i];
    gw[b * P + i] = (r > 0.0f) ? gl : ((r < 0.0f) ? -gl : 0.0f);
  }
}

static int check_img(const void *a, const void *b2, int B, int h, int w, const char *fn) {
  HG_REQUIRE(B >= 0, "%s: B < 0", fn);
  HG_REQUIRE(h >= 1 && w >= 1 && h <= 32768 && w <= 32768 &&
                 static_cast<int64_t>(h) * w <= (int64_t(1) << 29),
             "%s: image size %d x %d out of range", fn, h, w);
  if (B == 0) return HG_OK;
  HG_REQUIRE(a && b2, "%s: NULL pointer", fn);
  return HG_OK;
}

// General quadrilaterals (the tensorised general ACA): src, dst B x 8 floats
// (x_M y_M x_N y_N x_P y_P x_Q y_Q); H B x 9 doubles at ACA's own scale.
__global__ void aca_fwd_kernel(const float *__restrict__ src, const float *__restrict__ dst,
                               int B, double *__restrict__ H) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double s[8], d[8], h[9];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    s[k] = static_cast<double>(src[8 * b + k]);
    d[k] = static_cast<double>(dst[8 * b + k]);
  }
  (void)aca_solve(s, d, h);
#pragma unroll
  for (int i = 0; i < 9; ++i) H[9 * b + i] = h[i];
}

__global__ void aca_bwd_kernel(const float *__restrict__ src, const float *__restrict__ dst,
                               const double *__restrict__ gH, int B, float *__restrict__ gsrc,
                               float *__restrict__ gdst) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double s[8], d[8], g[9], gs[8], gd[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    s[k] = static_cast<double>(src[8 * b + k]);
    d[k] = static_cast<double>(dst[8 * b + k]);
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) g[i] = gH[9 * b + i];
  aca_vjp(s, d, g, gs, gd);
  if (gsrc) {
#pragma unroll
    for (int k = 0; k < 8; ++k) gsrc[8 * b + k] = static_cast<float>(gs[k]);
  }
  if (gdst) {
#pragma unroll
    for (int k = 0; k < 8; ++k) gdst[8 * b + k] = static_cast<float>(gd[k]);
  }
}

// Iterative refinement of the offsets (the six-solve structure of iterative
// deep homography networks, with the network's predicted update replaced by a
// gradient step on the photometric loss): per iteration one fused launch runs
// Algorithm 1, the warp + L1 backward, Algorithm 1's reverse mode and
// off -= step * grad for every patch.
struct RefineArgs {
  const float *img, *tgt;
  int B, h, w, iters;
  float step;
  float *off, *loss;
};

// The patch rectangle as hg_aca_rect_fwd receives it from a caller that
// passes w - 1 and (w - 1) / (h - 1) as floats.
static RectArgs patch_rect(int h, int w) {
  RectArgs ra;
  ra.x0 = 0.0;
  ra.y0 = 0.0;
  ra.w = static_cast<double>(static_cast<float>(w - 1));
  ra.r = static_cast<double>(static_cast<float>(double(w - 1) / double(h - 1)));
  return ra;
}

// Threads per patch workgroup: enough for about WAVES waves in flight over the
// batch, from 256 threads up to MAXNT. The forward kernels aim at 8192 waves
// (32 per CU) with up to 1024 threads; the backward ones at 4096 with up to
// 512 (they would spill registers at 1024, and more waves did not help them).
static int diff_threads(int B, int max_nt, int waves) {
  const int64_t want = (int64_t(waves) * 64 + B - 1) / std::max(B, 1);
  const int nt = want <= 256 ? 256 : want <= 512 ? 512 : 1024;
  return std::min(nt, max_nt);
}

template <int MAXNT = 1024, int WAVES = 8192, typename F>
static void with_threads(int B, F &&f) {
  const int nt = diff_threads(B, MAXNT, WAVES);
  if constexpr (MAXNT >= 1024) {
    if (nt == 1024) {
      f(std::integral_constant<int, 1024>());
      return;
    }
  }
  if (nt == 512) {
    f(std::integral_constant<int, 512>());
    return;
  }
  f(std::integral_constant<int, 256>());
}

static int launch_refine(const RefineArgs &a, hipStream_t s) {
  const RectArgs ra = patch_rect(a.h, a.w);
  for (int it = 0; it < a.iters; ++it) {
    with_threads<512, 4096>(a.B, [&](auto nt) {
      constexpr int NT = decltype(nt)::value;
      hipLaunchKernelGGL((photo_bwd_kernel<true, NT>), dim3(a.B), dim3(NT), 0, s, a.off, a.img,
                         a.tgt, nullptr, a.h, a.w, ra, a.step, nullptr);
    });
    if (int st = launched("photo_bwd_kernel<step>")) return st;
  }
  if (a.loss) {
    with_threads(a.B, [&](auto nt) {
      constexpr int NT = decltype(nt)::value;
      hipLaunchKernelGGL((photo_fwd_kernel<NT>), dim3(a.B), dim3(NT), 0, s, a.off, a.img, a.tgt,
                         a.h, a.w, ra, a.loss);
    });
    if (int st = launched("photo_fwd_kernel")) return st;
  }
  return HG_OK;
}

static int make_refine(const float *img, const float *tgt, int32_t B, int32_t h, int32_t w,
                       int32_t iters, float step, float *offsets, float *loss, const char *fn,
                       RefineArgs &a) {
  HG_REQUIRE(B >= 0, "%s: B < 0", fn);
  HG_REQUIRE(h >= 2 && w >= 2 && h <= 32768 && w <= 32768 &&
                 static_cast<int64_t>(h) * w <= (int64_t(1) << 29),
             "%s: image size %d x %d out of range", fn, h, w);
  HG_REQUIRE(iters >= 0 && iters <= 1000, "%s: iters = %d outside [0, 1000]", fn, iters);
  HG_REQUIRE(std::isfinite(step), "%s: step is not finite", fn);
  if (B > 0) HG_REQUIRE(img && tgt && offsets, "%s: NULL img, tgt or offsets", fn);
  a.img = img;
  a.tgt = tgt;
  a.B = B;
  a.h = h;
  a.w = w;
  a.iters = iters;
  a.step = step;
  a.off = offsets;
  a.loss = loss;
  return HG_OK;
}

static int check_rect(float w, float r, int B, const char *fn) {
  HG_REQUIRE(B >= 0, "%s: B < 0", fn);
  HG_REQUIRE(std::isfinite(w) && w > 0.0f && std::isfinite(r) && r > 0.0f,
             "%s: rectangle width and aspect ratio must be finite and > 0", fn);
  return HG_OK;
}

}  // namespace hg

using namespace hg;

extern "C" int hg_aca_rect_fwd(const float *offsets, int32_t B, float x0, float y0, float w,
                               float r, double *H, void *stream) {
  clear_error();
  if (int st = check_rect(w, r, B, "hg_aca_rect_fwd")) return st;
  if (B == 0) return HG_OK;
  HG_REQUIRE(offsets && H, "hg_aca_rect_fwd: NULL pointer");
  HG_REQUIRE(std::isfinite(x0) && std::isfinite(y0), "hg_aca_rect_fwd: non-finite origin");
  hipLaunchKernelGGL(rect_fwd_kernel, dim3((B + 255) / 256), dim3(256), 0, as_stream(stream),
                     offsets, B, static_cast<double>(x0), static_cast<double>(y0),
                     static_cast<double>(w), static_cast<double>(r), H);
  return launched("rect_fwd_kernel");
}

extern "C" int hg_aca_rect_bwd(const float *offsets, const double *grad_H, int32_t B, float x0,
                               float y0, float w, float r, float *grad_offsets, void *stream) {
  clear_error();
  if (int st = check_rect(w, r, B, "hg_aca_rect_bwd")) return st;
  if (B == 0) return HG_OK;
  HG_REQUIRE(offsets && grad_H && grad_offsets, "hg_aca_rect_bwd: NULL pointer");
  HG_REQUIRE(std::isfinite(x0) && std::isfinite(y0), "hg_aca_rect_bwd: non-finite origin");
  hipLaunchKernelGGL(rect_bwd_kernel, dim3((B + 255) / 256), dim3(256), 0, as_stream(stream),
                     offsets, grad_H, B, static_cast<double>(x0), static_cast<double>(y0),
                     static_cast<double>(w), static_cast<double>(r), grad_offsets);
  return launched("rect_bwd_kernel");
}

extern "C" int hg_aca_fwd(const float *src, const float *dst, int32_t B, double *H,
                          void *stream) {
  clear_error();
  HG_REQUIRE(B >= 0, "hg_aca_fwd: B < 0");
  if (B == 0) return HG_OK;
  HG_REQUIRE(src && dst && H, "hg_aca_fwd: NULL pointer");
  hipLaunchKernelGGL(aca_fwd_kernel, dim3((B + 255) / 256), dim3(256), 0, as_stream(stream), src,
                     dst, B, H);
  return launched("aca_fwd_kernel");
}

extern "C" int hg_aca_bwd(const float *src, const float *dst, const double *grad_H, int32_t B,
                          float *grad_src, float *grad_dst, void *stream) {
  clear_error();
  HG_REQUIRE(B >= 0, "hg_aca_bwd: B < 0");
  if (B == 0) return HG_OK;
  HG_REQUIRE(src && dst && grad_H, "hg_aca_bwd: NULL src, dst or grad_H");
  HG_REQUIRE(grad_src || grad_dst, "hg_aca_bwd: both gradient outputs are NULL");
  hipLaunchKernelGGL(aca_bwd_kernel, dim3((B + 255) / 256), dim3(256), 0, as_stream(stream), src,
                     dst, grad_H, B, grad_src, grad_dst);
  return launched("aca_bwd_kernel");
}

extern "C" int hg_warp_l1_fwd(const double *H, const float *img, const float *tgt, int32_t B,
                              int32_t h, int32_t w, float *loss, void *stream) {
  clear_error();
  if (int st = check_img(img, tgt, B, h, w, "hg_warp_l1_fwd")) return st;
  if (B == 0) return HG_OK;
  HG_REQUIRE(H && loss, "hg_warp_l1_fwd: NULL pointer");
  with_threads(B, [&](auto nt) {
    constexpr int NT = decltype(nt)::value;
    hipLaunchKernelGGL((warp_fwd_kernel<0, NT>), dim3(B), dim3(NT), 0, as_stream(stream), H, img,
                       tgt, h, w, loss, nullptr);
  });
  return launched("warp_fwd_kernel");
}

extern "C" int hg_warp_l1_bwd(const double *H, const float *img, const float *tgt,
                              const float *grad_loss, int32_t B, int32_t h, int32_t w,
                              double *grad_H, void *stream) {
  clear_error();
  if (int st = check_img(img, tgt, B, h, w, "hg_warp_l1_bwd")) return st;
  if (B == 0) return HG_OK;
  HG_REQUIRE(H && grad_loss && grad_H, "hg_warp_l1_bwd: NULL pointer");
  with_threads<512, 4096>(B, [&](auto nt) {
    constexpr int NT = decltype(nt)::value;
    hipLaunchKernelGGL((warp_bwd_kernel<false, NT>), dim3(B), dim3(NT), 0, as_stream(stream), H,
                       img, tgt, grad_loss, nullptr, h, w, grad_H);
  });
  return launched("warp_bwd_kernel");
}

extern "C" int hg_warp_store_fwd(const double *H, const float *img, int32_t B, int32_t h,
                                 int32_t w, float *warped, void *stream) {
  clear_error();
  if (int st = check_img(img, warped, B, h, w, "hg_warp_store_fwd")) return st;
  if (B == 0) return HG_OK;
  HG_REQUIRE(H, "hg_warp_store_fwd: NULL H");
  with_threads(B, [&](auto nt) {
    constexpr int NT = decltype(nt)::value;
    hipLaunchKernelGGL((warp_fwd_kernel<2, NT>), dim3(B), dim3(NT), 0, as_stream(stream), H, img,
                       nullptr, h, w, nullptr, warped);
  });
  return launched("warp_fwd_kernel<store>");
}

extern "C" int hg_l1_fwd(const float *warped, const float *tgt, int32_t B, int32_t h, int32_t w,
                         float *loss, void *stream) {
  clear_error();
  if (int st = check_img(warped, tgt, B, h, w, "hg_l1_fwd")) return st;
  if (B == 0) return HG_OK;
  HG_REQUIRE(loss, "hg_l1_fwd: NULL loss");
  hipLaunchKernelGGL(l1_fwd_kernel, dim3(B), dim3(kDiffThreads), 0, as_stream(stream), warped, tgt,
                     static_cast<int64_t>(h) * w, loss);
  return launched("l1_fwd_kernel");
}

extern "C" int hg_l1_bwd(const float *warped, const float *tgt, const float *grad_loss, int32_t B,
                         int32_t h, int32_t w, float *grad_warped, void *stream) {
  clear_error();
  if (int st = check_img(warped, tgt, B, h, w, "hg_l1_bwd")) return st;
  if (B == 0) return HG_OK;
  HG_REQUIRE(grad_loss && grad_warped, "hg_l1_bwd: NULL pointer");
  hipLaunchKernelGGL(l1_bwd_kernel, dim3(B), dim3(kDiffThreads), 0, as_stream(stream), warped, tgt,
                     grad_loss, static_cast<int64_t>(h) * w, grad_warped);
  return launched("l1_bwd_kernel");
}

extern "C" int hg_warp_bwd_from_grad(const double *H, const float *img, const float *grad_warped,
                                     int32_t B, int32_t h, int32_t w, double *grad_H,
                                     void *stream) {
  clear_error();
  if (int st = check_img(img, grad_warped, B, h, w, "hg_warp_bwd_from_grad")) return st;
  if (B == 0) return HG_OK;
  HG_REQUIRE(H && grad_H, "hg_warp_bwd_from_grad: NULL pointer");
  with_threads<512, 4096>(B, [&](auto nt) {
    constexpr int NT = decltype(nt)::value;
    hipLaunchKernelGGL((warp_bwd_kernel<true, NT>), dim3(B), dim3(NT), 0, as_stream(stream), H,
                       img, nullptr, nullptr, grad_warped, h, w, grad_H);
  });
  return launched("warp_bwd_kernel<stored>");
}

extern "C" int hg_photometric_fwd(const float *offsets, const float *img, const float *tgt,
                                  int32_t B, int32_t h, int32_t w, float *loss, void *stream) {
  clear_error();
  if (int st = check_img(img, tgt, B, h, w, "hg_photometric_fwd")) return st;
  HG_REQUIRE(h >= 2 && w >= 2, "hg_photometric_fwd: patches need h, w >= 2");
  if (B == 0) return HG_OK;
  HG_REQUIRE(offsets && loss, "hg_photometric_fwd: NULL offsets or loss");
  with_threads(B, [&](auto nt) {
    constexpr int NT = decltype(nt)::value;
    hipLaunchKernelGGL((photo_fwd_kernel<NT>), dim3(B), dim3(NT), 0, as_stream(stream), offsets,
                       img, tgt, h, w, patch_rect(h, w), loss);
  });
  return launched("photo_fwd_kernel");
}

extern "C" int hg_photometric_bwd(const float *offsets, const float *img, const float *tgt,
                                  const float *grad_loss, int32_t B, int32_t h, int32_t w,
                                  float *grad_offsets, void *stream) {
  clear_error();
  if (int st = check_img(img, tgt, B, h, w, "hg_photometric_bwd")) return st;
  HG_REQUIRE(h >= 2 && w >= 2, "hg_photometric_bwd: patches need h, w >= 2");
  if (B == 0) return HG_OK;
  HG_REQUIRE(offsets && grad_loss && grad_offsets, "hg_photometric_bwd: NULL pointer");
  with_threads<512, 4096>(B, [&](auto nt) {
    constexpr int NT = decltype(nt)::value;
    hipLaunchKernelGGL((photo_bwd_kernel<false, NT>), dim3(B), dim3(NT), 0, as_stream(stream),
                       const_cast<float *>(offsets), img, tgt, grad_loss, h, w, patch_rect(h, w),
                       0.0f, grad_offsets);
  });
  return launched("photo_bwd_kernel");
}

extern "C" int hg_refine(const float *img, const float *tgt, int32_t B, int32_t h, int32_t w,
                         int32_t iters, float step, float *offsets, float *loss, void *stream) {
  clear_error();
  RefineArgs a;
  if (int st = make_refine(img, tgt, B, h, w, iters, step, offsets, loss, "hg_refine", a))
    return st;
  if (B == 0) return HG_OK;
  return launch_refine(a, as_stream(stream));
}

extern "C" int hg_refine_graph_create(const float *img, const float *tgt, int32_t B, int32_t h,
                                      int32_t w, int32_t iters, float step, float *offsets,
                                      float *loss, void *stream, hg_graph **out) {
  clear_error();
  HG_REQUIRE(out, "hg_refine_graph_create: NULL out");
  *out = nullptr;
  RefineArgs a;
  if (int st = make_refine(img, tgt, B, h, w, iters, step, offsets, loss,
                           "hg_refine_graph_create", a))
    return st;
  HG_REQUIRE(B > 0, "hg_refine_graph_create: B must be > 0");
  return capture_graph(stream, [&](hipStream_t cap) { return launch_refine(a, cap); }, out);
}
