// Differentiable 4-point-offset pipeline: offsets -> H (ACA with the source
// corners fixed at a rectangle's) -> bilinear inverse warp -> L1 loss, with
// hand-written backward kernels that recompute per-pixel state from H, and a
// single-pass kernel that computes the loss and its gradient together.
//
// H and G = adj(H) are double precision, and so is each pixel's sample
// position: q = G (x, y, 1) and the projective division, whose reciprocal is
// a float estimate refined by one double Newton step (relative error ~2^-46,
// ~1e-12 px at patch scale). The floor that picks the bilinear cell is taken
// on that position, so cell choices (the kinks of the sampler) are those of
// float64 arithmetic. Everything after the floor runs in float: the bilinear
// weights (the cell fractions rounded to float), taps, residual, sign and the
// gradient terms; per-thread float partial sums are folded into double every
// 16 pixels, and per-patch sums across the workgroup are double.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "lanes.hpp"
#include "solver_dev.hpp"

namespace hg {

constexpr int kDiffThreads = 256;

// A rectangle with upper-left (x0, y0), width w and aspect ratio r = width /
// height, as ACA's source points M N P Q = TL, TR, BL, BR.
struct RectArgs {
  double x0, y0, w, r;
};

__device__ __forceinline__ void rect_source(const RectArgs &ra, double s[8]) {
  const double x1 = ra.x0 + ra.w, y1 = ra.y0 + ra.w / ra.r;
  s[0] = ra.x0;
  s[1] = ra.y0;
  s[2] = x1;
  s[3] = ra.y0;
  s[4] = ra.x0;
  s[5] = y1;
  s[6] = x1;
  s[7] = y1;
}

// Target points M N P Q = source corners + offsets (offset order TL TR BR BL).
__device__ __forceinline__ void rect_target(const float *o, const double s[8], double d[8]) {
  d[0] = s[0] + static_cast<double>(o[0]);
  d[1] = s[1] + static_cast<double>(o[1]);
  d[2] = s[2] + static_cast<double>(o[2]);
  d[3] = s[3] + static_cast<double>(o[3]);
  d[6] = s[6] + static_cast<double>(o[4]);
  d[7] = s[7] + static_cast<double>(o[5]);
  d[4] = s[4] + static_cast<double>(o[6]);
  d[5] = s[5] + static_cast<double>(o[7]);
}

// H (row-major, ACA's own scale) of one patch from its offsets.
__device__ __forceinline__ void rect_h(const float *o, const RectArgs &ra, double H[9]) {
  double s[8], d[8];
  rect_source(ra, s);
  rect_target(o, s, d);
  (void)aca_solve(s, d, H);
}

// dL/d offsets (order TL TR BR BL) from dL/dH, through ACA's reverse mode
// with respect to the target points.
__device__ __forceinline__ void rect_h_vjp(const float *o, const RectArgs &ra, const double gH[9],
                                           double g[8]) {
  double s[8], d[8], gs[8], gd[8];
  rect_source(ra, s);
  rect_target(o, s, d);
  aca_vjp(s, d, gH, gs, gd);
  g[0] = gd[0];
  g[1] = gd[1];
  g[2] = gd[2];
  g[3] = gd[3];
  g[4] = gd[6];
  g[5] = gd[7];
  g[6] = gd[4];
  g[7] = gd[5];
}

__global__ void rect_fwd_kernel(const float *__restrict__ off, int B, RectArgs ra,
                                double *__restrict__ H) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double h[9];
  rect_h(off + 8 * b, ra, h);
#pragma unroll
  for (int i = 0; i < 9; ++i) H[9 * b + i] = h[i];
}

__global__ void rect_bwd_kernel(const float *__restrict__ off, const double *__restrict__ gH, int B,
                                RectArgs ra, float *__restrict__ goff) {
  const int bi = blockIdx.x * blockDim.x + threadIdx.x;
  if (bi >= B) return;
  double g[8];
  rect_h_vjp(off + 8 * bi, ra, gH + 9 * bi, g);
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
// h w floats. The hardware checks a raw buffer load's range per dword: a dword
// at a byte offset at or past the buffer's end reads 0 without touching
// memory, also when it is the second half of an 8-byte load whose first half
// is inside. Each row of the cell is one 8-byte load of two adjacent floats
// starting at column cp = max(x0, 0) of the row, from which the taps x0 and
// x0 + 1 are picked and masked where they lie outside the image (at x0 = w - 1
// the second float is the next row's first, or past the end: masked). A row
// above the image gets an offset past the end; a row below it lies past the
// end already. Offsets are 32-bit and never negative.
constexpr uint32_t kFarOffset = 0x80000000u;   // past every patch (h w <= 2^29 floats)

struct TapAddr {
  uint32_t o0, o1;               // byte offsets of the column pair in rows y0, y0 + 1
  bool x0in, x1in;               // tap columns inside the image (x0 outside: x0 + 1 is
                                 // the pair's first float)
  float ax, ay;                  // fractional position in the cell
};

// Buffer over the P floats of one patch (P <= 2^29, so 4 P <= 2^31 bytes).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t patch_buffer(const float *I, int P) {
  return __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float *>(I), 0, static_cast<int>(static_cast<uint32_t>(P) * 4u), 0x00020000);
}

// Position clamped into [-2, w + 1] x [-2, h + 1] first (nan to -2): a cell
// it moves has all four taps outside before and after, and the cell indices
// stay small (h, w <= 32768). A row above the image gives a row offset that
// wraps past 2^31 as an unsigned number and is replaced by kFarOffset; rows
// at or below h lie at or past the buffer's end: both read 0. A cell with both
// columns outside (ix < -1 or ix >= w, so 0 <= cp <= w + 1) takes rows -4 and
// -3, whose offsets 4 (cp - 4 w) and 4 (cp - 3 w) are negative for every
// w >= 1: it reads no memory. Otherwise -1 <= ix < w and tap x0 exists iff
// ix >= 0, x0 + 1 iff ix <= w - 2.
__device__ __forceinline__ TapAddr tap_addr(double sx, double sy, int h, int w) {
  sx = fmin(fmax(sx, -2.0), static_cast<double>(w + 1));
  sy = fmin(fmax(sy, -2.0), static_cast<double>(h + 1));
  const double fx = floor(sx), fy = floor(sy);
  TapAddr t;
  t.ax = static_cast<float>(sx - fx);
  t.ay = static_cast<float>(sy - fy);
  const int ix = static_cast<int>(fx), iy = static_cast<int>(fy);
  const int cp = max(ix, 0);
  const int w4 = 4 * w;
  const bool cols = static_cast<uint32_t>(ix + 1) <= static_cast<uint32_t>(w);   // -1 <= ix < w
  uint32_t o = static_cast<uint32_t>(__mul24(cols ? iy : -4, w4) + 4 * cp);
  // the second row's offset is the first's plus one row (kept as one add:
  // without this the compiler recomputes it from cp with two more operations)
  asm volatile("" : "+v"(o));
  t.o0 = min(o, kFarOffset);
  t.o1 = min(o + static_cast<uint32_t>(w4), kFarOffset);
  t.x0in = ix >= 0;
  t.x1in = ix <= w - 2;
  return t;
}

// The column pairs of a cell's two rows, as loaded (rows outside read 0).
struct TapRaw {
  decltype(__builtin_amdgcn_raw_buffer_load_b64(__amdgpu_buffer_rsrc_t(), 0, 0, 0)) p0, p1;
};

__device__ __forceinline__ TapRaw tap_load(__amdgpu_buffer_rsrc_t r, const TapAddr &t) {
  TapRaw q;
  q.p0 = __builtin_amdgcn_raw_buffer_load_b64(r, t.o0, 0, 0);
  q.p1 = __builtin_amdgcn_raw_buffer_load_b64(r, t.o1, 0, 0);
  return q;
}

// The four taps of a cell (x0 y0, x1 y0, x0 y1, x1 y1; column-masked) from
// its loaded column pairs: the pair is (x0, x0 + 1), or (x0 + 1, x0 + 2) when
// x0 = -1 lies outside.
__device__ __forceinline__ void tap_pick(const TapAddr &t, const TapRaw &q, float L[4]) {
  const float a0 = __uint_as_float(q.p0[0]), b0 = __uint_as_float(q.p0[1]);
  const float a1 = __uint_as_float(q.p1[0]), b1 = __uint_as_float(q.p1[1]);
  L[0] = t.x0in ? a0 : 0.0f;
  L[1] = t.x1in ? (t.x0in ? b0 : a0) : 0.0f;
  L[2] = t.x0in ? a1 : 0.0f;
  L[3] = t.x1in ? (t.x0in ? b1 : a1) : 0.0f;
}

// Bilinear value and (GRAD) its derivatives in x and y inside the cell.
struct Tap {
  float v, dvdx, dvdy;
};

template <bool GRAD>
__device__ __forceinline__ Tap tap_eval(const TapAddr &a, const float L[4]) {
  const float d0 = L[1] - L[0], d1 = L[3] - L[2];
  const float top = fmaf(a.ax, d0, L[0]);
  const float bot = fmaf(a.ax, d1, L[2]);
  const float dy = bot - top;
  Tap t;
  t.v = fmaf(a.ay, dy, top);
  t.dvdx = 0.0f;
  t.dvdy = 0.0f;
  if (GRAD) {
    t.dvdx = fmaf(a.ay, d1 - d0, d0);
    t.dvdy = dy;
  }
  return t;
}

// 1/q: a float reciprocal estimate and one double Newton step (relative error
// ~2^-46; q outside the float range gives a non-finite position, which
// samples as outside the image).
__device__ __forceinline__ double recip(double q) {
  const double r = static_cast<double>(__builtin_amdgcn_rcpf(static_cast<float>(q)));
  return fma(fma(-q, r, 1.0), r, r);
}

// Pixels per thread per loop iteration (loads of all of them in flight at once).
constexpr int kUnroll = 4;
// Iterations between folds of the per-thread float partial sums into double.
constexpr int kFold = 4;

// Per-thread pixels (NT threads): pixel i = threadIdx.x + u NT + k NT kUnroll.
// ALIGNED (NT a multiple of w): all of a thread's pixels lie in one column
// x = threadIdx.x % w, each kUnroll-step k advancing every row by NT kUnroll / w;
// q = G (x, y, 1) is then a per-thread constant plus y G[:, 1] (3 FMAs).
// Otherwise (x, y) is walked per pixel and q takes 6 FMAs.
// ALIGNED keeps each row index as an exact float (rows < 2^24): that is the
// row of the float gradient sums as it stands, and one conversion gives the
// double row of q. Otherwise x and y are integers.
template <int NT, bool ALIGNED>
struct PixelWalk {
  int x[kUnroll], y[kUnroll];
  float yf[kUnroll];
  int step_x, step_y, w;
  __device__ __forceinline__ PixelWalk(int w_) : w(w_) {
    constexpr int kStep = NT * kUnroll;
    step_y = kStep / w;
    step_x = kStep % w;
    if (ALIGNED) {
      // one column per thread: pixel threadIdx.x + u NT is NT / w rows below
      // pixel threadIdx.x + (u - 1) NT
      const int y0 = static_cast<int>(threadIdx.x) / w;
      const int x0 = static_cast<int>(threadIdx.x) - y0 * w;
      const int dy = NT / w;
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        y[u] = y0 + u * dy;
        x[u] = x0;
        yf[u] = static_cast<float>(y[u]);
      }
    } else {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int i = static_cast<int>(threadIdx.x) + u * NT;
        y[u] = i / w;
        x[u] = i % w;
      }
    }
  }
  __device__ __forceinline__ double row_d(int u) const {
    return ALIGNED ? static_cast<double>(yf[u]) : static_cast<double>(y[u]);
  }
  __device__ __forceinline__ float row_f(int u) const {
    return ALIGNED ? yf[u] : static_cast<float>(y[u]);
  }
  __device__ __forceinline__ void advance() {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (ALIGNED) {
        yf[u] += static_cast<float>(step_y);
      } else {
        y[u] += step_y;
        x[u] += step_x;
        if (x[u] >= w) {
          x[u] -= w;
          ++y[u];
        }
      }
    }
  }
};

// Workgroup (NT threads) sum of NV per-thread partials, in double. Result valid
// in thread 0. The partials go through LDS: lane (k, r) of the first NV x 16
// threads adds the partials r, r + 16, r + 32, ... of value k in that order,
// then the 16 lanes of value k (one DPP row) add their sums in row order. A
// fixed order, so the result is deterministic; the DPP work is one row scan
// per value instead of one per value and thread row.
template <int NV, int NT>
__device__ __forceinline__ void block_sum(const double (&v)[NV], double (&out)[NV]) {
  constexpr int kParts = 16;
  static_assert(NV * kParts <= NT && NT % kParts == 0, "16 lanes per value");
  __shared__ double part[NV][NT];
  __shared__ double tot[NV];
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NV; ++k) part[k][t] = v[k];
  __syncthreads();
  if (t < NV * kParts) {
    const int k = t / kParts, r = t % kParts;
    double x = part[k][r];
#pragma unroll
    for (int j = 1; j < NT / kParts; ++j) x += part[k][j * kParts + r];
    x = row_sum16_f64(x);
    if (r == kParts - 1) tot[k] = x;
  }
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = tot[k];
  }
}

// Per-patch G = 2^-e adj(H) shared by the workgroup, read back into scalar
// registers (it is uniform).
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

// What a per-patch warp pass computes.
enum WarpMode {
  kLoss = 0,        // loss[b] = mean |I_w - T|
  kGrad = 1,        // dL/dH from sign(r) gl, gl = grad_loss[b] / (h w) (recomputed r)
  kStore = 2,       // warped image, rounded to float
  kGradStored = 3,  // dL/dH from a stored dL/dI_w
  kLossGrad = 4,    // loss[b] and dloss[b]/dH in one pass (gl = 1 / (h w))
};

// One patch b per workgroup; Hb: its 9 entries of H (global or LDS). Writes
// the loss (kLoss, kLossGrad; thread 0), the warped image (kStore), and dL/dH
// to gHout (kGrad, kGradStored, kLossGrad; thread 0, 9 doubles).
// The gradient of the loss through q = G p, position (q0, q1) / q2: with
// g = dL/dI_w at a pixel (gl sign(r) for the L1 loss, gl a per-patch
// constant), (a0, a1) = g iq grad I there and iq = 1/q2,
// dL/dG row 1 += a0 p, row 2 += a1 p, row 3 += -(a0 sx + a1 sy) p.
template <int MODE, int NT, bool ALIGNED>
__device__ __forceinline__ void warp_block(const double *Hb, const float *__restrict__ img,
                                           const float *__restrict__ tgt, float gl, int h, int w,
                                           int b, float *__restrict__ loss,
                                           float *__restrict__ warped, double *gHout) {
  constexpr bool GRAD = MODE == kGrad || MODE == kGradStored || MODE == kLossGrad;
  constexpr bool LOSS = MODE == kLoss || MODE == kLossGrad;
  double G[9];
  int e;
  load_G(Hb, G, e);
  const int P = h * w;
  const __amdgpu_buffer_rsrc_t rs = patch_buffer(img + static_cast<int64_t>(b) * P, P);
  // the second stream (target or stored gradient) as a buffer too: indices
  // past the patch (the last loop's tail) read 0
  const float *T2 = MODE == kStore ? img : tgt;
  const __amdgpu_buffer_rsrc_t rt = patch_buffer(T2 + static_cast<int64_t>(b) * P, P);
  // float partial sums (folded every kFold iterations) and their double totals:
  // 0..8 the dL/dG terms, 9 the loss. ALIGNED: x is the thread's column, so the
  // x-multiplied sums 0, 3, 6 are x times the sums 2, 5, 8, taken at the fold
  constexpr int NS = 10;
  float sf[NS];
  double sd[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    sf[k] = 0.0f;
    sd[k] = 0.0;
  }
  PixelWalk<NT, ALIGNED> pw(w);
  // ALIGNED: per-thread constant part of q (column x)
  double A[3] = {0.0, 0.0, 0.0};
  const float xcol = static_cast<float>(pw.x[0]);
  if (ALIGNED) {
    const double xd = static_cast<double>(pw.x[0]);
#pragma unroll
    for (int r = 0; r < 3; ++r) A[r] = fma(G[3 * r], xd, G[3 * r + 2]);
  }
  auto fold = [&]() {
    if (ALIGNED) {
#pragma unroll
      for (int k = 0; k < 9; k += 3)
        sd[k] += static_cast<double>(sf[k + 2]) * static_cast<double>(xcol);
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      if (ALIGNED && (k == 0 || k == 3 || k == 6)) continue;
      sd[k] += static_cast<double>(sf[k]);
      sf[k] = 0.0f;
    }
  };
  // one iteration of kUnroll pixels per thread; TAIL: the last, partly past
  // the patch
  auto iteration = [&](int i0, auto tail_tag) {
    constexpr bool TAIL = decltype(tail_tag)::value;
    TapAddr ta[kUnroll];
    TapRaw raw[kUnroll];
    float tv[kUnroll], sxf[kUnroll], syf[kUnroll], iqf[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const double yd = pw.row_d(u);
      double q0, q1, q2;
      if (ALIGNED) {
        q0 = fma(G[1], yd, A[0]);
        q1 = fma(G[4], yd, A[1]);
        q2 = fma(G[7], yd, A[2]);
      } else {
        const double xd = static_cast<double>(pw.x[u]);
        q0 = fma(G[0], xd, fma(G[1], yd, G[2]));
        q1 = fma(G[3], xd, fma(G[4], yd, G[5]));
        q2 = fma(G[6], xd, fma(G[7], yd, G[8]));
      }
      const double iq = recip(q2);
      const double sx = q0 * iq, sy = q1 * iq;
      ta[u] = tap_addr(sx, sy, h, w);
      if (TAIL && i0 + u * NT >= P) ta[u].o0 = ta[u].o1 = kFarOffset;   // past the patch: 0
      if (GRAD) {
        sxf[u] = static_cast<float>(sx);
        syf[u] = static_cast<float>(sy);
        iqf[u] = static_cast<float>(iq);
      }
      raw[u] = tap_load(rs, ta[u]);
      if (MODE != kStore)
        tv[u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
            rt, static_cast<uint32_t>(i0 + u * NT) * 4u, 0, 0));
    }
    // every pixel's loads are issued before the first is used
    __builtin_amdgcn_sched_barrier(0);
    // TAIL: a pixel past the patch read 0 for its taps and its target
    // (r = 0) and is masked out of the gradient without a branch, so that no
    // pixel's loads move into a conditional block
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int i = i0 + u * NT;
      const bool in = !TAIL || i < P;
      float L[4];
      tap_pick(ta[u], raw[u], L);
      const Tap t = tap_eval<GRAD>(ta[u], L);
      if (MODE == kStore && in) warped[static_cast<int64_t>(b) * P + i] = t.v;
      const float r = t.v - tv[u];
      if (LOSS) sf[9] += fabsf(r);
      if (GRAD) {
        // g iq
        float gi;
        if (MODE == kGradStored) {
          gi = tv[u] * iqf[u];
        } else {
          // gl iq sign(r), with sign(0) = 0 (and 0 for a nan residual)
          const float gq = gl * iqf[u];
          gi = fabsf(r) > 0.0f ? copysignf(gq, r) : 0.0f;
        }
        gi = in ? gi : 0.0f;
        const float a0 = gi * t.dvdx, a1 = gi * t.dvdy;
        const float na2 = fmaf(a0, sxf[u], a1 * syf[u]);   // -(row 3 term)
        const float yf = pw.row_f(u);
        if (!ALIGNED) {
          const float xf = static_cast<float>(pw.x[u]);
          sf[0] = fmaf(a0, xf, sf[0]);
          sf[3] = fmaf(a1, xf, sf[3]);
          sf[6] = fmaf(-na2, xf, sf[6]);
        }
        sf[1] = fmaf(a0, yf, sf[1]);
        sf[2] += a0;
        sf[4] = fmaf(a1, yf, sf[4]);
        sf[5] += a1;
        sf[7] = fmaf(-na2, yf, sf[7]);
        sf[8] -= na2;
      }
    }
  };
  // full iterations (every pixel of the workgroup inside the patch), then at
  // most one partial one; the fold cadence is per iteration
  // The workgroups of one batch are resident together and have equal work,
  // but the waves' issue arbitration favours some of them, which finish early
  // and leave their slots idle while the rest run on a thinner CU. Each wave's
  // priority therefore steps down as it advances (3 in the first quarter of
  // its iterations, 0 in the last), so that waves behind are issued first.
  const int n_full = P / (NT * kUnroll);
  int since = 0, it = 0, prio = 3;
  __builtin_amdgcn_s_setprio(3);
  int i0 = threadIdx.x;
  for (; i0 - static_cast<int>(threadIdx.x) + NT * kUnroll <= P; i0 += NT * kUnroll) {
    const int want = 3 - (4 * it) / max(n_full, 1);
    if (want != prio) {
      prio = want;
      if (want == 2) __builtin_amdgcn_s_setprio(2);
      else if (want == 1) __builtin_amdgcn_s_setprio(1);
      else __builtin_amdgcn_s_setprio(0);
    }
    iteration(i0, std::false_type());
    pw.advance();
    ++it;
    if (++since == kFold) {
      fold();
      since = 0;
    }
  }
  if (i0 - static_cast<int>(threadIdx.x) < P) iteration(i0, std::true_type());
  __builtin_amdgcn_s_setprio(0);
  fold();
  if (LOSS && !GRAD) {
    double s1[1] = {sd[9]}, o1[1];
    block_sum<1, NT>(s1, o1);
    if (threadIdx.x == 0) loss[b] = static_cast<float>(o1[0] / static_cast<double>(P));
  }
  if (GRAD) {
    double s10[NS], o10[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) s10[k] = sd[k];
    block_sum<NS, NT>(s10, o10);
    if (threadIdx.x == 0) {
      if (LOSS) loss[b] = static_cast<float>(o10[9] / static_cast<double>(P));
      adjugate_backward(Hb, o10, e, gHout);
    }
  }
}

// Per-pixel kernels: at least 4 waves per SIMD (at most 128 VGPRs).
template <int MODE, int NT, bool ALIGNED>
__global__ __launch_bounds__(NT, 4) void warp_kernel(const double *__restrict__ H,
                                                  const float *__restrict__ img,
                                                  const float *__restrict__ tgt,
                                                  const float *__restrict__ grad_loss, int h,
                                                  int w, float *__restrict__ loss,
                                                  float *__restrict__ warped,
                                                  double *__restrict__ grad_H) {
  const int b = blockIdx.x;
  const float gl = MODE == kGrad ? static_cast<float>(static_cast<double>(grad_loss[b]) /
                                                      static_cast<double>(h * w))
                                 : 0.0f;
  warp_block<MODE, NT, ALIGNED>(H + 9 * b, img, tgt, gl, h, w, b, loss, warped, grad_H + 9 * b);
}

// ---- fused offsets -> loss / gradient (one workgroup per patch) -------------
// ACA with the rectangle's source corners runs in thread 0 of the patch's
// workgroup into LDS, then the warp; gradients go back through ACA's reverse
// mode in thread 0. The arithmetic is that of the separate kernels.
// Only thread 0 reads Hs (load_G and adjugate_backward run in it), so no
// barrier follows; load_G's barrier then publishes G to the workgroup.
__device__ __forceinline__ void rect_to_lds(const float *o, const RectArgs &ra, double *Hs) {
  if (threadIdx.x == 0) {
    double hh[9];
    rect_h(o, ra, hh);
#pragma unroll
    for (int i = 0; i < 9; ++i) Hs[i] = hh[i];
  }
}

template <int NT, bool ALIGNED>
__global__ __launch_bounds__(NT, 4) void photo_fwd_kernel(const float *__restrict__ off,
                                                       const float *__restrict__ img,
                                                       const float *__restrict__ tgt, int h,
                                                       int w, RectArgs ra,
                                                       float *__restrict__ loss) {
  __shared__ double Hs[9];
  rect_to_lds(off + 8 * blockIdx.x, ra, Hs);
  warp_block<kLoss, NT, ALIGNED>(Hs, img, tgt, 0.0f, h, w, blockIdx.x, loss, nullptr, nullptr);
}

// grad_offsets = grad_loss[b] dL_b/d offsets_b; with STEP, instead
// offsets_b -= step * float(dL_b/d offsets_b) in place (grad_loss = 1).
template <bool STEP, int NT, bool ALIGNED>
__global__ __launch_bounds__(NT, 4) void photo_bwd_kernel(
    float *__restrict__ off, const float *__restrict__ img, const float *__restrict__ tgt,
    const float *__restrict__ grad_loss, int h, int w, RectArgs ra, float step,
    float *__restrict__ goff) {
  __shared__ double Hs[9];
  __shared__ double gHs[9];
  const int b = blockIdx.x;
  rect_to_lds(off + 8 * b, ra, Hs);
  const float gl = static_cast<float>(static_cast<double>(STEP ? 1.0f : grad_loss[b]) /
                                      static_cast<double>(h * w));
  warp_block<kGrad, NT, ALIGNED>(Hs, img, tgt, gl, h, w, b, nullptr, nullptr, gHs);
  if (threadIdx.x == 0) {
    double g[8];
    rect_h_vjp(off + 8 * b, ra, gHs, g);
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

// Loss and its gradient in one pass over img and tgt: loss[b] and
// grad_unit[b] = dloss[b]/d offsets_b (grad_loss = 1).
template <int NT, bool ALIGNED>
__global__ __launch_bounds__(NT, 4) void photo_fwd_grad_kernel(
    const float *__restrict__ off, const float *__restrict__ img, const float *__restrict__ tgt,
    int h, int w, RectArgs ra, float *__restrict__ loss, float *__restrict__ grad_unit) {
  __shared__ double Hs[9];
  __shared__ double gHs[9];
  const int b = blockIdx.x;
  rect_to_lds(off + 8 * b, ra, Hs);
  const float gl = static_cast<float>(1.0 / static_cast<double>(h * w));
  warp_block<kLossGrad, NT, ALIGNED>(Hs, img, tgt, gl, h, w, b, loss, nullptr, gHs);
  if (threadIdx.x == 0) {
    double g[8];
    rect_h_vjp(off + 8 * b, ra, gHs, g);
#pragma unroll
    for (int i = 0; i < 8; ++i) grad_unit[8 * b + i] = static_cast<float>(g[i]);
  }
}

// out[b, k] = grad_loss[b] * grad_unit[b, k] (8 per patch).
__global__ void scale_grad_kernel(const float *__restrict__ grad_unit,
                                  const float *__restrict__ grad_loss, int B,
                                  float *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 8 * B) out[i] = grad_loss[i / 8] * grad_unit[i];
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

// Most patches per call (32-bit per-patch offsets such as 9 B stay in range).
constexpr int32_t kMaxPatches = 1 << 27;

static int check_img(const void *a, const void *b2, int B, int h, int w, const char *fn) {
  HG_REQUIRE(B >= 0 && B <= kMaxPatches, "%s: B = %d outside [0, 2^27]", fn, B);
  HG_REQUIRE(h >= 1 && w >= 1 && h <= 32768 && w <= 32768 &&
                 static_cast<int64_t>(h) * w <= (int64_t(1) << 29),
             "%s: image size %d x %d out of range", fn, h, w);
  if (B == 0) return HG_OK;
  HG_REQUIRE(a && b2, "%s: NULL pointer", fn);
  return HG_OK;
}

// General quadrilaterals (the tensorised general ACA): src, dst B x 8 floats
// (x_M y_M x_N y_N x_P y_P x_Q y_Q); H B x 9 doubles at ACA's own scale.
// One problem per thread, kDiffThreads per workgroup. The 9 doubles of each
// H go through LDS, so that the workgroup's block of H (9 kDiffThreads
// doubles, contiguous) is written as consecutive doubles: every store
// instruction covers 512 contiguous bytes instead of lanes 72 bytes apart.
__global__ __launch_bounds__(kDiffThreads) void aca_fwd_kernel(const float *__restrict__ src,
                                                               const float *__restrict__ dst,
                                                               int B, double *__restrict__ H) {
  __shared__ double hs[9 * kDiffThreads];
  const int b0 = blockIdx.x * kDiffThreads;
  const int b = b0 + threadIdx.x;
  if (b < B) {
    double s[8], d[8], h[9];
    const int64_t o = 8 * static_cast<int64_t>(b);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      s[k] = static_cast<double>(src[o + k]);
      d[k] = static_cast<double>(dst[o + k]);
    }
    (void)aca_solve(s, d, h);
#pragma unroll
    for (int i = 0; i < 9; ++i) hs[9 * threadIdx.x + i] = h[i];
  }
  __syncthreads();
  const int nd = 9 * min(kDiffThreads, B - b0);   // doubles of this workgroup's block
  double *Hb = H + 9 * static_cast<int64_t>(b0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int k = i * kDiffThreads + threadIdx.x;
    if (k < nd) Hb[k] = hs[k];
  }
}

__global__ void aca_bwd_kernel(const float *__restrict__ src, const float *__restrict__ dst,
                               const double *__restrict__ gH, int B, float *__restrict__ gsrc,
                               float *__restrict__ gdst) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double s[8], d[8], g[9], gs[8], gd[8];
  const int64_t o = 8 * static_cast<int64_t>(b), oh = 9 * static_cast<int64_t>(b);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    s[k] = static_cast<double>(src[o + k]);
    d[k] = static_cast<double>(dst[o + k]);
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) g[i] = gH[oh + i];
  aca_vjp(s, d, g, gs, gd);
  if (gsrc) {
#pragma unroll
    for (int k = 0; k < 8; ++k) gsrc[o + k] = static_cast<float>(gs[k]);
  }
  if (gdst) {
#pragma unroll
    for (int k = 0; k < 8; ++k) gdst[o + k] = static_cast<float>(gd[k]);
  }
}

// Iterative refinement of the offsets (the six-solve structure of iterative
// deep homography networks, with the network's predicted update replaced by a
// gradient step on the photometric loss): per iteration one fused launch runs
// ACA with the rectangle's source corners, the warp + L1 backward, ACA's reverse mode and
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

// Launch shape of a per-patch kernel: f(NT, ALIGNED) with NT from
// diff_threads and ALIGNED = (NT is a multiple of the patch width w).
template <int MAXNT = 1024, int WAVES = 8192, typename F>
static void with_shape(int B, int w, F &&f) {
  const int nt = diff_threads(B, MAXNT, WAVES);
  const bool al = nt % w == 0;
  auto go = [&](auto NTc) {
    if (al)
      f(NTc, std::true_type());
    else
      f(NTc, std::false_type());
  };
  if constexpr (MAXNT >= 1024) {
    if (nt == 1024) {
      go(std::integral_constant<int, 1024>());
      return;
    }
  }
  if (nt == 512) {
    go(std::integral_constant<int, 512>());
    return;
  }
  go(std::integral_constant<int, 256>());
}

static int launch_refine(const RefineArgs &a, hipStream_t s) {
  const RectArgs ra = patch_rect(a.h, a.w);
  for (int it = 0; it < a.iters; ++it) {
    with_shape<512, 4096>(a.B, a.w, [&](auto nt, auto al) {
      constexpr int NT = decltype(nt)::value;
      constexpr bool AL = decltype(al)::value;
      hipLaunchKernelGGL((photo_bwd_kernel<true, NT, AL>), dim3(a.B), dim3(NT), 0, s, a.off,
                         a.img, a.tgt, nullptr, a.h, a.w, ra, a.step, nullptr);
    });
    if (int st = launched("photo_bwd_kernel<step>")) return st;
  }
  if (a.loss) {
    with_shape(a.B, a.w, [&](auto nt, auto al) {
      constexpr int NT = decltype(nt)::value;
      constexpr bool AL = decltype(al)::value;
      hipLaunchKernelGGL((photo_fwd_kernel<NT, AL>), dim3(a.B), dim3(NT), 0, s, a.off, a.img,
                         a.tgt, a.h, a.w, ra, a.loss);
    });
    if (int st = launched("photo_fwd_kernel")) return st;
  }
  return HG_OK;
}

static int make_refine(const float *img, const float *tgt, int32_t B, int32_t h, int32_t w,
                       int32_t iters, float step, float *offsets, float *loss, const char *fn,
                       RefineArgs &a) {
  HG_REQUIRE(B >= 0 && B <= kMaxPatches, "%s: B = %d outside [0, 2^27]", fn, B);
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
  HG_REQUIRE(B >= 0 && B <= kMaxPatches, "%s: B = %d outside [0, 2^27]", fn, B);
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
  const RectArgs ra = {static_cast<double>(x0), static_cast<double>(y0), static_cast<double>(w),
                       static_cast<double>(r)};
  hipLaunchKernelGGL(rect_fwd_kernel, dim3((B + 255) / 256), dim3(256), 0, as_stream(stream),
                     offsets, B, ra, H);
  return launched("rect_fwd_kernel");
}

extern "C" int hg_aca_rect_bwd(const float *offsets, const double *grad_H, int32_t B, float x0,
                               float y0, float w, float r, float *grad_offsets, void *stream) {
  clear_error();
  if (int st = check_rect(w, r, B, "hg_aca_rect_bwd")) return st;
  if (B == 0) return HG_OK;
  HG_REQUIRE(offsets && grad_H && grad_offsets, "hg_aca_rect_bwd: NULL pointer");
  HG_REQUIRE(std::isfinite(x0) && std::isfinite(y0), "hg_aca_rect_bwd: non-finite origin");
  const RectArgs ra = {static_cast<double>(x0), static_cast<double>(y0), static_cast<double>(w),
                       static_cast<double>(r)};
  hipLaunchKernelGGL(rect_bwd_kernel, dim3((B + 255) / 256), dim3(256), 0, as_stream(stream),
                     offsets, grad_H, B, ra, grad_offsets);
  return launched("rect_bwd_kernel");
}

extern "C" int hg_aca_fwd(const float *src, const float *dst, int32_t B, double *H,
                          void *stream) {
  clear_error();
  HG_REQUIRE(B >= 0 && B <= (1 << 30), "hg_aca_fwd: B = %d outside [0, 2^30]", B);
  if (B == 0) return HG_OK;
  HG_REQUIRE(src && dst && H, "hg_aca_fwd: NULL pointer");
  hipLaunchKernelGGL(aca_fwd_kernel, dim3((B + kDiffThreads - 1) / kDiffThreads), dim3(kDiffThreads),
                     0, as_stream(stream), src, dst, B, H);
  return launched("aca_fwd_kernel");
}

extern "C" int hg_aca_bwd(const float *src, const float *dst, const double *grad_H, int32_t B,
                          float *grad_src, float *grad_dst, void *stream) {
  clear_error();
  HG_REQUIRE(B >= 0 && B <= (1 << 30), "hg_aca_bwd: B = %d outside [0, 2^30]", B);
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
  with_shape(B, w, [&](auto nt, auto al) {
    constexpr int NT = decltype(nt)::value;
    constexpr bool AL = decltype(al)::value;
    hipLaunchKernelGGL((warp_kernel<kLoss, NT, AL>), dim3(B), dim3(NT), 0, as_stream(stream), H,
                       img, tgt, nullptr, h, w, loss, nullptr, nullptr);
  });
  return launched("warp_kernel<loss>");
}

extern "C" int hg_warp_l1_bwd(const double *H, const float *img, const float *tgt,
                              const float *grad_loss, int32_t B, int32_t h, int32_t w,
                              double *grad_H, void *stream) {
  clear_error();
  if (int st = check_img(img, tgt, B, h, w, "hg_warp_l1_bwd")) return st;
  if (B == 0) return HG_OK;
  HG_REQUIRE(H && grad_loss && grad_H, "hg_warp_l1_bwd: NULL pointer");
  with_shape<512, 4096>(B, w, [&](auto nt, auto al) {
    constexpr int NT = decltype(nt)::value;
    constexpr bool AL = decltype(al)::value;
    hipLaunchKernelGGL((warp_kernel<kGrad, NT, AL>), dim3(B), dim3(NT), 0, as_stream(stream), H,
                       img, tgt, grad_loss, h, w, nullptr, nullptr, grad_H);
  });
  return launched("warp_kernel<grad>");
}

extern "C" int hg_warp_store_fwd(const double *H, const float *img, int32_t B, int32_t h,
                                 int32_t w, float *warped, void *stream) {
  clear_error();
  if (int st = check_img(img, warped, B, h, w, "hg_warp_store_fwd")) return st;
  if (B == 0) return HG_OK;
  HG_REQUIRE(H, "hg_warp_store_fwd: NULL H");
  with_shape(B, w, [&](auto nt, auto al) {
    constexpr int NT = decltype(nt)::value;
    constexpr bool AL = decltype(al)::value;
    hipLaunchKernelGGL((warp_kernel<kStore, NT, AL>), dim3(B), dim3(NT), 0, as_stream(stream), H,
                       img, nullptr, nullptr, h, w, nullptr, warped, nullptr);
  });
  return launched("warp_kernel<store>");
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
  with_shape<512, 4096>(B, w, [&](auto nt, auto al) {
    constexpr int NT = decltype(nt)::value;
    constexpr bool AL = decltype(al)::value;
    hipLaunchKernelGGL((warp_kernel<kGradStored, NT, AL>), dim3(B), dim3(NT), 0,
                       as_stream(stream), H, img, grad_warped, nullptr, h, w, nullptr, nullptr,
                       grad_H);
  });
  return launched("warp_kernel<grad_stored>");
}

extern "C" int hg_photometric_fwd(const float *offsets, const float *img, const float *tgt,
                                  int32_t B, int32_t h, int32_t w, float *loss, void *stream) {
  clear_error();
  if (int st = check_img(img, tgt, B, h, w, "hg_photometric_fwd")) return st;
  HG_REQUIRE(h >= 2 && w >= 2, "hg_photometric_fwd: patches need h, w >= 2");
  if (B == 0) return HG_OK;
  HG_REQUIRE(offsets && loss, "hg_photometric_fwd: NULL offsets or loss");
  with_shape(B, w, [&](auto nt, auto al) {
    constexpr int NT = decltype(nt)::value;
    constexpr bool AL = decltype(al)::value;
    hipLaunchKernelGGL((photo_fwd_kernel<NT, AL>), dim3(B), dim3(NT), 0, as_stream(stream),
                       offsets, img, tgt, h, w, patch_rect(h, w), loss);
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
  with_shape<512, 4096>(B, w, [&](auto nt, auto al) {
    constexpr int NT = decltype(nt)::value;
    constexpr bool AL = decltype(al)::value;
    hipLaunchKernelGGL((photo_bwd_kernel<false, NT, AL>), dim3(B), dim3(NT), 0, as_stream(stream),
                       const_cast<float *>(offsets), img, tgt, grad_loss, h, w, patch_rect(h, w),
                       0.0f, grad_offsets);
  });
  return launched("photo_bwd_kernel");
}

extern "C" int hg_photometric_fwd_grad(const float *offsets, const float *img, const float *tgt,
                                       int32_t B, int32_t h, int32_t w, float *loss,
                                       float *grad_unit, void *stream) {
  clear_error();
  if (int st = check_img(img, tgt, B, h, w, "hg_photometric_fwd_grad")) return st;
  HG_REQUIRE(h >= 2 && w >= 2, "hg_photometric_fwd_grad: patches need h, w >= 2");
  if (B == 0) return HG_OK;
  HG_REQUIRE(offsets && loss && grad_unit, "hg_photometric_fwd_grad: NULL pointer");
  with_shape<512, 4096>(B, w, [&](auto nt, auto al) {
    constexpr int NT = decltype(nt)::value;
    constexpr bool AL = decltype(al)::value;
    hipLaunchKernelGGL((photo_fwd_grad_kernel<NT, AL>), dim3(B), dim3(NT), 0, as_stream(stream),
                       offsets, img, tgt, h, w, patch_rect(h, w), loss, grad_unit);
  });
  return launched("photo_fwd_grad_kernel");
}

extern "C" int hg_scale_grad(const float *grad_unit, const float *grad_loss, int32_t B,
                             float *grad_offsets, void *stream) {
  clear_error();
  HG_REQUIRE(B >= 0, "hg_scale_grad: B < 0");
  if (B == 0) return HG_OK;
  HG_REQUIRE(grad_unit && grad_loss && grad_offsets, "hg_scale_grad: NULL pointer");
  HG_REQUIRE(B <= (1 << 27), "hg_scale_grad: B too large");
  hipLaunchKernelGGL(scale_grad_kernel, dim3((8 * B + 255) / 256), dim3(256), 0,
                     as_stream(stream), grad_unit, grad_loss, B, grad_offsets);
  return launched("scale_grad_kernel");
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
