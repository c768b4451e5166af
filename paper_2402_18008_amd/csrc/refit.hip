// n-point homography refit on RANSAC inliers by the HO-SVD reduction (the
// paper's recommendation for n points): both sides are normalised about their
// centroids with an isotropic scale giving RMS distance sqrt(2); the first
// two rows of H are eliminated in the least-squares sense, leaving the last
// row h3 as the right singular vector of the 2n x 3 matrix
//   M = [(I - P) D_u X ; (I - P) D_v X],   X = [x y 1], P = X (X^T X)^-1 X^T,
// and h1 = (X^T X)^-1 X^T D_u X h3, h2 likewise with D_v.
//
// One workgroup per pair, one pass over the points (batches of 8 per thread,
// loads issued ahead of use): the count and 29 moments of the coordinates
// taken relative to the pair's first point, summed in double. One lane shifts
// them to the centroids (binomial expansion: every moment needed for the shift
// is among the 30 sums), the normalisation enters as powers of the two
// scales, and the same lane forms the 3 x 3 Gram matrix
//   M^T M = S2u - S1u S0^-1 S1u + S2v - S1v S0^-1 S1v
// (S0 = X^T X, S1u = X^T D_u X, S2u = X^T D_u^2 X), takes its eigenvector of
// smallest eigenvalue as the dominant eigenvector of its adjugate (repeated
// squaring; cyclic Jacobi rotations when the two smallest eigenvalues are too
// close for that to converge), recovers h1, h2,
// denormalises and writes the power-of-two scaled float H. Moments about a
// point of the pair rather than the origin keep the shift's cancellation to
// the ratio of that point's distance from the centroid to the spread; when the
// point lies more than 4 RMS spreads away (an unselected outlier), the
// moments are summed again about the centroid found.
#include <cmath>

#include "common.hpp"
#include "lanes.hpp"
#include "solver_dev.hpp"

namespace hg {

constexpr int kRefitThreads = 256;
constexpr int kMoments = 29;   // centred: S0 5 (and the count), S1u, S2u, S1v, S2v 6 each
constexpr int kRaw = 30;       // about the first point: 6 monomials each times 1, u, u^2, v, v^2

// Points are visited kBatch at a time per thread (i0 + j * kRefitThreads),
// all their loads issued before any is used: one memory round trip per batch
// instead of one per point. A thread's points keep their order, so the sums
// do not depend on kBatch.
constexpr int kBatch = 8;

struct PointBatch {
  float x1[kBatch], y1[kBatch], x2[kBatch], y2[kBatch];
  bool sel[kBatch];   // the point exists and its mask byte is set
};

__device__ __forceinline__ void load_batch(const float *X1, const float *Y1, const float *X2,
                                           const float *Y2, const uint8_t *mask, int64_t i0,
                                           int64_t b, PointBatch &pb) {
#pragma unroll
  for (int j = 0; j < kBatch; ++j) {
    const int64_t i = i0 + static_cast<int64_t>(j) * kRefitThreads;
    const bool in = i < b;
    const int64_t ic = in ? i : b - 1;   // i0 < b, so every load stays inside the pair
    pb.x1[j] = X1[ic];
    pb.y1[j] = Y1[ic];
    pb.x2[j] = X2[ic];
    pb.y2[j] = Y2[ic];
    pb.sel[j] = in && (!mask || mask[ic] != 0);
  }
}

// Workgroup sum of NV doubles; the result is valid in thread 0. Each row of 16
// lanes sums its values (row_sum16_f64), then thread k adds the rows' partials
// of value k in row order: a fixed order, so the result is deterministic.
template <int NV>
__device__ __forceinline__ void refit_block_sum(double (&v)[NV]) {
  constexpr int kRows = kRefitThreads / 16;
  static_assert(NV <= kRefitThreads, "one thread per value");
  __shared__ double red[NV][kRows];
  __shared__ double tot[NV];
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = row_sum16_f64(v[k]);
    if ((t & 15) == 15) red[k][t >> 4] = s;
  }
  __syncthreads();
  if (t < NV) {
    double s = red[t][0];
#pragma unroll
    for (int r = 1; r < kRows; ++r) s += red[t][r];
    tot[t] = s;
  }
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = tot[k];
  }
  __syncthreads();
}

// Symmetric 3 x 3 from the six monomial sums m = {xx, xy, x, yy, y, 1} with
// the scales a (source) applied as X = [a x, a y, 1] and a factor f.
__host__ __device__ __forceinline__ void sym3(const double *m, double a, double f, double S[3][3]) {
  S[0][0] = f * a * a * m[0];
  S[0][1] = S[1][0] = f * a * a * m[1];
  S[0][2] = S[2][0] = f * a * m[2];
  S[1][1] = f * a * a * m[3];
  S[1][2] = S[2][1] = f * a * m[4];
  S[2][2] = f * m[5];
}

__host__ __device__ __forceinline__ bool inverse3(const double A[3][3], double Ai[3][3]) {
  const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
  if (!(fabs(det) > 0.0) || !(fabs(det) <= 1.7976931348623157e308)) return false;
  const double r = 1.0 / det;
  Ai[0][0] = c00 * r;
  Ai[1][0] = c01 * r;
  Ai[2][0] = c02 * r;
  Ai[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * r;
  Ai[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * r;
  Ai[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * r;
  Ai[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * r;
  Ai[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * r;
  Ai[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * r;
  return true;
}

__host__ __device__ __forceinline__ void matmul3(const double A[3][3], const double B[3][3],
                                        double C[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[i][j] = A[i][0] * B[0][j] + A[i][1] * B[1][j] + A[i][2] * B[2][j];
}

// Cyclic Jacobi eigenvalue iteration on a symmetric 3 x 3 (Golub and Van
// Loan, Sec. 8.5): each rotation zeroes one off-diagonal entry; V collects the
// rotations (eigenvectors in its columns). Returns the column of the smallest
// eigenvalue in v.
__host__ __device__ inline void smallest_eigvec3(double A[3][3], double v[3]) {
  double V[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    // converged when the off-diagonal mass is at the rounding level of the
    // diagonal (eps^2 ~ 5e-32): further sweeps cannot reduce it
    if (!(off > 1e-30 * dia)) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      const double apq = A[p][q];
      if (apq == 0.0) continue;
      // rotation (c, s) with t = tan: t^2 + 2 tau t - 1 = 0, the smaller root
      const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
      const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
      const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
#pragma unroll
      for (int k = 0; k < 3; ++k) {   // A <- A J (columns p, q)
        const double akp = A[k][p], akq = A[k][q];
        A[k][p] = c * akp - s * akq;
        A[k][q] = s * akp + c * akq;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {   // A <- J^T A (rows p, q)
        const double apk = A[p][k], aqk = A[q][k];
        A[p][k] = c * apk - s * aqk;
        A[q][k] = s * apk + c * aqk;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {   // V <- V J
        const double vkp = V[k][p], vkq = V[k][q];
        V[k][p] = c * vkp - s * vkq;
        V[k][q] = s * vkp + c * vkq;
      }
    }
  }
  int m = 0;
  double am = A[0][0];
  if (A[1][1] < am) {
    m = 1;
    am = A[1][1];
  }
  if (A[2][2] < am) m = 2;
  // selects rather than a variable index, which would put V in scratch memory
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] = m == 0 ? V[k][0] : (m == 1 ? V[k][1] : V[k][2]);
}

// Eigenvector of the smallest eigenvalue of a symmetric positive
// semi-definite 3 x 3 C. Its adjugate has the same eigenvectors with the
// eigenvalues l2 l3, l1 l3 and l1 l2 (0 <= l1 <= l2 <= l3), so the wanted
// vector is adj(C)'s dominant one. Repeated squaring of adj(C) (rescaled to
// max |entry| = 1 each time) squares the ratio l1 / l2 at every step, so the
// matrix becomes rank one, every column parallel to the wanted vector; the
// column of largest norm is taken once it stops changing direction. If that
// does not happen within 12 squarings (l1 within ~0.1 % of l2: a
// near-degenerate problem) the Jacobi iteration decides.
__host__ __device__ inline void smallest_eigvec3_adj(const double C[3][3], double v[3]) {
  double A[3][3];
  A[0][0] = C[1][1] * C[2][2] - C[1][2] * C[2][1];
  A[0][1] = C[0][2] * C[2][1] - C[0][1] * C[2][2];
  A[0][2] = C[0][1] * C[1][2] - C[0][2] * C[1][1];
  A[1][1] = C[0][0] * C[2][2] - C[0][2] * C[2][0];
  A[1][2] = C[0][2] * C[1][0] - C[0][0] * C[1][2];
  A[2][2] = C[0][0] * C[1][1] - C[0][1] * C[1][0];
  A[1][0] = A[0][1];
  A[2][0] = A[0][2];
  A[2][1] = A[1][2];
  double x[3] = {0.0, 0.0, 0.0};
  bool ok = false;
  for (int it = 0; it < 13; ++it) {
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) m = fmax(m, fabs(A[i / 3][i % 3]));
    if (!(m > 0.0) || !(m <= 1.7976931348623157e308)) break;
    const double r = 1.0 / m;
#pragma unroll
    for (int i = 0; i < 9; ++i) A[i / 3][i % 3] *= r;
    // column of largest norm, scaled to max |component| = 1
    int k = 0;
    double best = -1.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double s = A[0][j] * A[0][j] + A[1][j] * A[1][j] + A[2][j] * A[2][j];
      if (s > best) {
        best = s;
        k = j;
      }
    }
    double y[3] = {A[0][k], A[1][k], A[2][k]};
    const double my = fmax(fabs(y[0]), fmax(fabs(y[1]), fabs(y[2])));
    // orient like the previous estimate, then compare directions
    double dot = y[0] * x[0] + y[1] * x[1] + y[2] * x[2];
    const double sg = dot < 0.0 ? -1.0 / my : 1.0 / my;
    double d = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      y[i] *= sg;
      d = fmax(d, fabs(y[i] - x[i]));
      x[i] = y[i];
    }
    if (it > 0 && d <= 1e-14) {
      ok = true;
      break;
    }
    double S[3][3];
    matmul3(A, A, S);
#pragma unroll
    for (int i = 0; i < 9; ++i) A[i / 3][i % 3] = S[i / 3][i % 3];
  }
  if (!ok) {
    double Cj[3][3];
#pragma unroll
    for (int i = 0; i < 9; ++i) Cj[i / 3][i % 3] = C[i / 3][i % 3];
    smallest_eigvec3(Cj, v);
    return;
  }
  const double r = 1.0 / sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] = x[i] * r;
}

// Sums of the monomials {xx, xy, x, yy, y, 1} of x - a, y - b from those of
// x, y (same weights).
__host__ __device__ __forceinline__ void shift6(const double *r, double a, double b, double *c) {
  c[0] = r[0] - 2.0 * a * r[2] + a * a * r[5];
  c[1] = r[1] - b * r[2] - a * r[4] + a * b * r[5];
  c[2] = r[2] - a * r[5];
  c[3] = r[3] - 2.0 * b * r[4] + b * b * r[5];
  c[4] = r[4] - b * r[5];
  c[5] = r[5];
}

// Centred moments m (layout of refit_solve) and the centroids' offsets from the
// reference point, from the sums r about it: r[0..5] the monomials of (x, y),
// r[6..11] u times them, r[12..17] u^2 times them, r[18..23] and r[24..29] the
// same for v; r[5] is the count (> 0). With u = u' - c:
// sum u M = sum u' M - c sum M and sum u^2 M = sum u'^2 M - 2 c sum u' M + c^2 sum M.
__host__ __device__ inline void center_moments(const double *r, double *m, double &a, double &b,
                                               double &c, double &d) {
  const double n = r[5];
  a = r[2] / n;
  b = r[4] / n;
  c = r[11] / n;
  d = r[23] / n;
  double m0[6], mu1[6], mu2[6], mv1[6], mv2[6];
  shift6(r, a, b, m0);
  shift6(r + 6, a, b, mu1);
  shift6(r + 12, a, b, mu2);
  shift6(r + 18, a, b, mv1);
  shift6(r + 24, a, b, mv2);
#pragma unroll
  for (int k = 0; k < 5; ++k) m[k] = m0[k];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    m[5 + k] = mu1[k] - c * m0[k];
    m[11 + k] = mu2[k] - 2.0 * c * mu1[k] + c * c * m0[k];
    m[17 + k] = mv1[k] - d * m0[k];
    m[23 + k] = mv2[k] - 2.0 * d * mv1[k] + d * d * m0[k];
  }
}

// The per-pair solve from the centred moments m (layout: S0's {xx, xy, x, yy,
// y}, then u, u^2, v, v^2 times {xx, xy, x, yy, y, 1}), the count n and the
// centroids: H (row-major, double) = T2^-1 Hn T1,
// or zeros when X^T X is singular.
__host__ __device__ inline void refit_solve(const double *m, double n, double cx, double cy,
                                            double cu, double cv, double *h) {
  // scales: RMS distance sqrt(2) on each side
  const double sa = sqrt(2.0 * n / (m[0] + m[3]));
  const double sb = sqrt(2.0 * n / (m[16] + m[28]));
  const double m0[6] = {m[0], m[1], m[2], m[3], m[4], n};
  double S0[3][3], S1u[3][3], S2u[3][3], S1v[3][3], S2v[3][3], S0i[3][3];
  sym3(m0, sa, 1.0, S0);
  sym3(m + 5, sa, sb, S1u);
  sym3(m + 11, sa, sb * sb, S2u);
  sym3(m + 17, sa, sb, S1v);
  sym3(m + 23, sa, sb * sb, S2v);
  bool ok = inverse3(S0, S0i);
  if (ok) {
    double Tu[3][3], Tv[3][3], Pu[3][3], Pv[3][3];
    matmul3(S0i, S1u, Tu);   // S0^-1 S1u
    matmul3(S0i, S1v, Tv);
    matmul3(S1u, Tu, Pu);    // S1u S0^-1 S1u
    matmul3(S1v, Tv, Pv);
    double C[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) C[i][j] = (S2u[i][j] - Pu[i][j]) + (S2v[i][j] - Pv[i][j]);
    // symmetrise against rounding
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i + 1; j < 3; ++j) C[i][j] = C[j][i] = 0.5 * (C[i][j] + C[j][i]);
    double h3[3];
    smallest_eigvec3_adj(C, h3);
    double Hn[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Hn[0][j] = Tu[j][0] * h3[0] + Tu[j][1] * h3[1] + Tu[j][2] * h3[2];
      Hn[1][j] = Tv[j][0] * h3[0] + Tv[j][1] * h3[1] + Tv[j][2] * h3[2];
      Hn[2][j] = h3[j];
    }
    // H = T2^-1 Hn T1, T1 = [[sa, 0, -sa cx], [0, sa, -sa cy], [0, 0, 1]],
    // T2^-1 = [[1/sb, 0, cu], [0, 1/sb, cv], [0, 0, 1]]
    const double T1[3][3] = {{sa, 0.0, -sa * cx}, {0.0, sa, -sa * cy}, {0.0, 0.0, 1.0}};
    const double T2i[3][3] = {{1.0 / sb, 0.0, cu}, {0.0, 1.0 / sb, cv}, {0.0, 0.0, 1.0}};
    double A[3][3], Hd[3][3];
    matmul3(T2i, Hn, A);
    matmul3(A, T1, Hd);
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = Hd[i / 3][i % 3];
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = 0.0;
  }
}

__global__ __launch_bounds__(kRefitThreads) void refit_kernel(
    const float *__restrict__ corr, int64_t ld, const int64_t *__restrict__ off,
    const uint8_t *__restrict__ mask, float *__restrict__ Hout, int32_t *__restrict__ n_used,
    uint8_t *__restrict__ flags) {
  const int p = blockIdx.x;
  // the pair's range, clamped into the planes
  const int64_t a = min(max(off[p], int64_t(0)), ld);
  const int64_t b = min(max(off[p + 1], a), ld);
  const float *X1 = corr, *Y1 = corr + ld, *X2 = corr + 2 * ld, *Y2 = corr + 3 * ld;
  // reference point: the pair's first point, selected or not; a coordinate
  // that is not finite there is replaced by 0, so that unselected points never
  // enter the sums
  double rx = 0.0, ry = 0.0, ru = 0.0, rv = 0.0;
  if (b > a) {
    rx = static_cast<double>(X1[a]);
    ry = static_cast<double>(Y1[a]);
    ru = static_cast<double>(X2[a]);
    rv = static_cast<double>(Y2[a]);
    rx = isfinite(rx) ? rx : 0.0;
    ry = isfinite(ry) ? ry : 0.0;
    ru = isfinite(ru) ? ru : 0.0;
    rv = isfinite(rv) ? rv : 0.0;
  }
  // the count and the 29 moments of the selected points about the reference
  // (workgroup sum in thread 0)
  double r[kRaw];
  auto moments = [&]() {
#pragma unroll
    for (int k = 0; k < kRaw; ++k) r[k] = 0.0;
    for (int64_t i0 = a + threadIdx.x; i0 < b; i0 += kRefitThreads * kBatch) {
      PointBatch pb;
      load_batch(X1, Y1, X2, Y2, mask, i0, b, pb);
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        if (!pb.sel[j]) continue;
        const double x = static_cast<double>(pb.x1[j]) - rx, y = static_cast<double>(pb.y1[j]) - ry;
        const double u = static_cast<double>(pb.x2[j]) - ru, v = static_cast<double>(pb.y2[j]) - rv;
        const double mono[6] = {x * x, x * y, x, y * y, y, 1.0};
        const double uu = u * u, vv = v * v;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          r[k] += mono[k];
          r[6 + k] += u * mono[k];
          r[12 + k] += uu * mono[k];
          r[18 + k] += v * mono[k];
          r[24 + k] += vv * mono[k];
        }
      }
    }
    refit_block_sum(r);
  };
  moments();
  // The shift to the centroids cancels about (distance / spread)^4 of the
  // fourth moments: a reference more than 4 RMS spreads from the centroid of
  // either side (an unselected outlier far from the rest) is replaced by the
  // centroid found, and the moments are summed again about it.
  __shared__ double again[5];
  if (threadIdx.x == 0) {
    const double n0 = r[5];
    bool far = false;
    if (n0 >= 4.0) {
      const double ma = r[2] / n0, mb = r[4] / n0, mc = r[11] / n0, md = r[23] / n0;
      const double s1 = (r[0] + r[3]) / n0 - (ma * ma + mb * mb);
      const double s2 = (r[17] + r[29]) / n0 - (mc * mc + md * md);
      far = !(ma * ma + mb * mb <= 16.0 * s1) || !(mc * mc + md * md <= 16.0 * s2);
      again[1] = rx + ma;
      again[2] = ry + mb;
      again[3] = ru + mc;
      again[4] = rv + md;
    }
    again[0] = far ? 1.0 : 0.0;
  }
  __syncthreads();
  if (again[0] != 0.0) {   // uniform across the workgroup
    rx = again[1];
    ry = again[2];
    ru = again[3];
    rv = again[4];
    moments();
  }
  if (threadIdx.x != 0) return;
  const double n = r[5];
  const int used = static_cast<int>(n);
  if (used < 4) {
#pragma unroll
    for (int k = 0; k < 9; ++k) Hout[9 * p + k] = 0.0f;
    if (n_used) n_used[p] = used;
    if (flags) flags[p] = static_cast<uint8_t>(kZeroH);
    return;
  }
  double m[kMoments], da, db, dc, dd;
  center_moments(r, m, da, db, dc, dd);
  const double cx = rx + da, cy = ry + db, cu = ru + dc, cv = rv + dd;
  double h[9];
  refit_solve(m, n, cx, cy, cu, cv, h);
  float hf[9];
  const uint32_t f = scale_to_float(h, hf);
#pragma unroll
  for (int k = 0; k < 9; ++k) Hout[9 * p + k] = hf[k];
  if (n_used) n_used[p] = used;
  if (flags) flags[p] = static_cast<uint8_t>(f);
}

}  // namespace hg

using namespace hg;

extern "C" int hg_refit_ho(const float *corr, int64_t ld, const int64_t *off, int32_t n_pairs,
                           const uint8_t *mask, float *H, int32_t *n_used, uint8_t *flags,
                           void *stream) {
  clear_error();
  HG_REQUIRE(n_pairs >= 0, "hg_refit_ho: n_pairs = %d < 0", n_pairs);
  if (n_pairs == 0) return HG_OK;
  HG_REQUIRE(corr && off && H, "hg_refit_ho: NULL corr, off or H");
  HG_REQUIRE(ld >= 1 && ld <= (INT64_MAX / 8), "hg_refit_ho: ld = %lld out of range",
             static_cast<long long>(ld));
  hipLaunchKernelGGL(refit_kernel, dim3(n_pairs), dim3(kRefitThreads), 0, as_stream(stream), corr,
                     ld, off, mask, H, n_used, flags);
  return launched("refit_kernel");
}
