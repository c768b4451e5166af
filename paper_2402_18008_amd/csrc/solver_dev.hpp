// Device functions for the minimal 4-point homography: ACA (Sec. 4) and SKS
// (Sec. 3), the degeneracy test and the power-of-two output scaling.
//
// Arithmetic is double precision on float inputs. The translation units are
// compiled with -ffp-contract=off, so every rounding is the one written here
// and every kernel that includes these functions produces bit-identical
// results for the same input.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hg {

constexpr uint32_t kNearDegenerate = 1u;  // a triangle of either side is thinner than kDelta
constexpr uint32_t kNonfiniteInput = 2u;
constexpr uint32_t kZeroH = 4u;           // H zero or non-finite: written as zeros
constexpr double kDelta = 1e-2;           // minimum admissible triangle height, px
constexpr double kDelta2 = kDelta * kDelta;

// Squared edge length between points i and j of one side.
__host__ __device__ __forceinline__ double edge2(const double *x, const double *y, int i, int j) {
  const double dx = x[j] - x[i];
  const double dy = y[j] - y[i];
  return dx * dx + dy * dy;
}

// True if one of the 4 triangles of a side has height <= kDelta over its
// longest edge: A^2 <= delta^2 * max(edge^2), with A the doubled signed area.
// The areas of MNP, MQP, MNQ and NPQ are exactly the ACA quantities f_A, Q.x,
// Q.y and t of that side (eqs. f_A_1, Q3, t1).
__host__ __device__ __forceinline__ bool side_thin(const double *x, const double *y, double aMNP,
                                          double aMQP, double aMNQ, double aNPQ) {
  const double mn = edge2(x, y, 0, 1), mp = edge2(x, y, 0, 2), mq = edge2(x, y, 0, 3);
  const double np = edge2(x, y, 1, 2), nq = edge2(x, y, 1, 3), pq = edge2(x, y, 2, 3);
  bool thin = aMNP * aMNP <= kDelta2 * fmax(fmax(mn, mp), np);
  thin |= aMQP * aMQP <= kDelta2 * fmax(fmax(mq, mp), pq);
  thin |= aMNQ * aMNQ <= kDelta2 * fmax(fmax(mn, mq), nq);
  thin |= aNPQ * aNPQ <= kDelta2 * fmax(fmax(np, nq), pq);
  return thin;
}

// ACA: H = H_A2^-1 H_C H_A1 up to scale, without division (Sec. 4, Table IV:
// 7 + 7 FLOPs for the affinities, 28 for the core, 10 + 33 for the product).
// s, d: x_M y_M x_N y_N x_P y_P x_Q y_Q of source and target. H row-major.
// Returns the near-degeneracy bit.
__host__ __device__ __forceinline__ uint32_t aca_solve(const double *s, const double *d,
                                                          double *H) {
  const double M1x = s[0], M1y = s[1], N1x = s[2], N1y = s[3];
  const double P1x = s[4], P1y = s[5], Q1x = s[6], Q1y = s[7];
  const double M2x = d[0], M2y = d[1], N2x = d[2], N2y = d[3];
  const double P2x = d[4], P2y = d[5], Q2x = d[6], Q2y = d[7];
  // H_A1 (eq. AffineExpresion): maps M1, N1, P1 to (0,0), (1,0), (0,1), weight f_A1
  const double MN1x = N1x - M1x, MN1y = N1y - M1y;
  const double MP1x = P1x - M1x, MP1y = P1y - M1y;
  const double fA1 = MN1x * MP1y - MN1y * MP1x;
  // H_A2 likewise on the target side
  const double MN2x = N2x - M2x, MN2y = N2y - M2y;
  const double MP2x = P2x - M2x, MP2y = P2y - M2y;
  const double fA2 = MN2x * MP2y - MN2y * MP2x;
  // fourth point under the affinities (eq. Q3) and the core (eqs. t1, C_11)
  const double MQ1x = Q1x - M1x, MQ1y = Q1y - M1y;
  const double MQ2x = Q2x - M2x, MQ2y = Q2y - M2y;
  const double Q3x = MQ1x * MP1y - MQ1y * MP1x;
  const double Q3y = MN1x * MQ1y - MN1y * MQ1x;
  const double Q4x = MQ2x * MP2y - MQ2y * MP2x;
  const double Q4y = MN2x * MQ2y - MN2y * MQ2x;
  const double t1 = fA1 - Q3x - Q3y;
  const double t2 = fA2 - Q4x - Q4y;
  const double c11 = t1 * Q3y * Q4x;
  const double c22 = t1 * Q3x * Q4y;
  const double c33 = t2 * Q3x * Q3y;
  // L = H_A2^-1 H_C: row 3 of H_C is (c11 - c33, c22 - c33, c33)
  const double mx = M2x * c33, my = M2y * c33;
  const double L[3][3] = {{N2x * c11 - mx, P2x * c22 - mx, mx},
                          {N2y * c11 - my, P2y * c22 - my, my},
                          {c11 - c33, c22 - c33, c33}};
  // H = L H_A1, H_A1 = [[MP1y, -MP1x, .], [-MN1y, MN1x, .], [0, 0, f_A1]] T(-M1)
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double h0 = L[i][0] * MP1y - L[i][1] * MN1y;
    const double h1 = L[i][1] * MN1x - L[i][0] * MP1x;
    H[3 * i + 0] = h0;
    H[3 * i + 1] = h1;
    H[3 * i + 2] = L[i][2] * fA1 - (h0 * M1x + h1 * M1y);
  }
  const double x1[4] = {M1x, N1x, P1x, Q1x}, y1[4] = {M1y, N1y, P1y, Q1y};
  const double x2[4] = {M2x, N2x, P2x, Q2x}, y2[4] = {M2y, N2y, P2y, Q2y};
  const bool thin = side_thin(x1, y1, fA1, Q3x, Q3y, t1) || side_thin(x2, y2, fA2, Q4x, Q4y, t2);
  return thin ? kNearDegenerate : 0u;
}

// Reverse mode of aca_solve: given gH = dL/dH (row-major, H at ACA's own
// scale), accumulate-free gs = dL/ds and gd = dL/dd (8 each, point order
// M N P Q). The forward quantities are recomputed, then each step of the
// forward order is differentiated in reverse: composition H = L H_A1, the
// product L = H_A2^-1 H_C, the core c11, c22, c33, the signed areas, and the
// difference vectors.
__host__ __device__ __forceinline__ void aca_vjp(const double *s, const double *d,
                                                 const double *gH, double *gs, double *gd) {
  const double M1x = s[0], M1y = s[1];
  const double M2x = d[0], M2y = d[1], N2x = d[2], N2y = d[3], P2x = d[4], P2y = d[5];
  const double MN1x = s[2] - M1x, MN1y = s[3] - M1y;
  const double MP1x = s[4] - M1x, MP1y = s[5] - M1y;
  const double MQ1x = s[6] - M1x, MQ1y = s[7] - M1y;
  const double MN2x = N2x - M2x, MN2y = N2y - M2y;
  const double MP2x = P2x - M2x, MP2y = P2y - M2y;
  const double MQ2x = d[6] - M2x, MQ2y = d[7] - M2y;
  const double fA1 = MN1x * MP1y - MN1y * MP1x;
  const double fA2 = MN2x * MP2y - MN2y * MP2x;
  const double Q3x = MQ1x * MP1y - MQ1y * MP1x;
  const double Q3y = MN1x * MQ1y - MN1y * MQ1x;
  const double Q4x = MQ2x * MP2y - MQ2y * MP2x;
  const double Q4y = MN2x * MQ2y - MN2y * MQ2x;
  const double t1 = fA1 - Q3x - Q3y;
  const double t2 = fA2 - Q4x - Q4y;
  const double c11 = t1 * Q3y * Q4x;
  const double c22 = t1 * Q3x * Q4y;
  const double c33 = t2 * Q3x * Q3y;
  const double mx = M2x * c33, my = M2y * c33;
  const double L[3][3] = {{N2x * c11 - mx, P2x * c22 - mx, mx},
                          {N2y * c11 - my, P2y * c22 - my, my},
                          {c11 - c33, c22 - c33, c33}};
  // H row i: h0 = L0 MP1y - L1 MN1y, h1 = L1 MN1x - L0 MP1x, h2 = L2 fA1 - (h0 M1x + h1 M1y)
  double gL[3][3];
  double gM1x = 0.0, gM1y = 0.0, gMN1x = 0.0, gMN1y = 0.0, gMP1x = 0.0, gMP1y = 0.0;
  double gfA1 = 0.0;
  for (int i = 0; i < 3; ++i) {
    const double h0 = L[i][0] * MP1y - L[i][1] * MN1y;
    const double h1 = L[i][1] * MN1x - L[i][0] * MP1x;
    const double g2 = gH[3 * i + 2];
    const double g0 = gH[3 * i + 0] - g2 * M1x;
    const double g1 = gH[3 * i + 1] - g2 * M1y;
    gM1x -= g2 * h0;
    gM1y -= g2 * h1;
    gL[i][2] = g2 * fA1;
    gfA1 += g2 * L[i][2];
    gL[i][0] = g0 * MP1y - g1 * MP1x;
    gL[i][1] = g1 * MN1x - g0 * MN1y;
    gMP1y += g0 * L[i][0];
    gMN1y -= g0 * L[i][1];
    gMN1x += g1 * L[i][1];
    gMP1x -= g1 * L[i][0];
  }
  // L = H_A2^-1 H_C
  const double gmx = gL[0][2] - gL[0][0] - gL[0][1];
  const double gmy = gL[1][2] - gL[1][0] - gL[1][1];
  const double gc11 = gL[0][0] * N2x + gL[1][0] * N2y + gL[2][0];
  const double gc22 = gL[0][1] * P2x + gL[1][1] * P2y + gL[2][1];
  const double gc33 = gL[2][2] - gL[2][0] - gL[2][1] + gmx * M2x + gmy * M2y;
  double gM2x = gmx * c33, gM2y = gmy * c33;
  const double gN2x = gL[0][0] * c11, gN2y = gL[1][0] * c11;
  const double gP2x = gL[0][1] * c22, gP2y = gL[1][1] * c22;
  // core
  const double gt1 = gc11 * Q3y * Q4x + gc22 * Q3x * Q4y;
  const double gt2 = gc33 * Q3x * Q3y;
  const double gQ3x = gc22 * t1 * Q4y + gc33 * t2 * Q3y - gt1;
  const double gQ3y = gc11 * t1 * Q4x + gc33 * t2 * Q3x - gt1;
  const double gQ4x = gc11 * t1 * Q3y - gt2;
  const double gQ4y = gc22 * t1 * Q3x - gt2;
  gfA1 += gt1;
  const double gfA2 = gt2;
  // signed areas: source side
  gMN1x += gfA1 * MP1y + gQ3y * MQ1y;
  gMN1y += -gfA1 * MP1x - gQ3y * MQ1x;
  gMP1x += -gfA1 * MN1y - gQ3x * MQ1y;
  gMP1y += gfA1 * MN1x + gQ3x * MQ1x;
  const double gMQ1x = gQ3x * MP1y - gQ3y * MN1y;
  const double gMQ1y = gQ3y * MN1x - gQ3x * MP1x;
  // target side
  const double gMN2x = gfA2 * MP2y + gQ4y * MQ2y;
  const double gMN2y = -gfA2 * MP2x - gQ4y * MQ2x;
  const double gMP2x = -gfA2 * MN2y - gQ4x * MQ2y;
  const double gMP2y = gfA2 * MN2x + gQ4x * MQ2x;
  const double gMQ2x = gQ4x * MP2y - gQ4y * MN2y;
  const double gMQ2y = gQ4y * MN2x - gQ4x * MP2x;
  // difference vectors
  gs[0] = gM1x - gMN1x - gMP1x - gMQ1x;
  gs[1] = gM1y - gMN1y - gMP1y - gMQ1y;
  gs[2] = gMN1x;
  gs[3] = gMN1y;
  gs[4] = gMP1x;
  gs[5] = gMP1y;
  gs[6] = gMQ1x;
  gs[7] = gMQ1y;
  gM2x -= gMN2x + gMP2x + gMQ2x;
  gM2y -= gMN2y + gMP2y + gMQ2y;
  gd[0] = gM2x;
  gd[1] = gM2y;
  gd[2] = gN2x + gMN2x;
  gd[3] = gN2y + gMN2y;
  gd[4] = gP2x + gMP2x;
  gd[5] = gP2y + gMP2y;
  gd[6] = gMQ2x;
  gd[7] = gMQ2y;
}

// Doubled signed areas (MNP, MQP, MNQ, NPQ) of one side, as in ACA.
__host__ __device__ __forceinline__ bool quad_side_thin(const double *q) {
  const double MNx = q[2] - q[0], MNy = q[3] - q[1];
  const double MPx = q[4] - q[0], MPy = q[5] - q[1];
  const double MQx = q[6] - q[0], MQy = q[7] - q[1];
  const double fA = MNx * MPy - MNy * MPx;
  const double Qx = MQx * MPy - MQy * MPx;
  const double Qy = MNx * MQy - MNy * MQx;
  const double t = fA - Qx - Qy;
  const double x[4] = {q[0], q[2], q[4], q[6]}, y[4] = {q[1], q[3], q[5], q[7]};
  return side_thin(x, y, fA, Qx, Qy, t);
}

// SKS: H = H_S2^-1 H_K H_S1 (Sec. 3). H_S maps the anchors M, N to (-1, 0) and
// (1, 0) (eq. 3_2_4); P and Q, mapped by H_S and the swap H_E, become P5, Q5
// (source) and P6, Q6 (target) as inhomogeneous points; the hyperbolic
// rotation-scale (a, b) solves eq. 4, whose sum and difference give a + b and
// a - b directly; u, v complete H_K (eq. H_K).
__device__ __forceinline__ uint32_t sks_solve(const double *s, const double *d, double *H) {
  // similarity parameters (eqs. 3_2_1, 3_2_2, fOfS1)
  const double ON1x = (s[2] - s[0]) * 0.5, ON1y = (s[3] - s[1]) * 0.5;
  const double O1x = s[0] + ON1x, O1y = s[1] + ON1y;
  const double f1 = ON1x * ON1x + ON1y * ON1y;
  const double ON2x = (d[2] - d[0]) * 0.5, ON2y = (d[3] - d[1]) * 0.5;
  const double O2x = d[0] + ON2x, O2y = d[1] + ON2y;
  const double f2 = ON2x * ON2x + ON2y * ON2y;
  auto canon = [](double Ox, double Oy, double ONx, double ONy, double px, double py,
                  double &cx, double &cy) {
    const double dx = px - Ox, dy = py - Oy;
    cx = ONx * dx + ONy * dy;
    cy = ONx * dy - ONy * dx;
  };
  double P3x, P3y, P4x, P4y, Q3x, Q3y, Q4x, Q4y;
  canon(O1x, O1y, ON1x, ON1y, s[4], s[5], P3x, P3y);
  canon(O2x, O2y, ON2x, ON2y, d[4], d[5], P4x, P4y);
  canon(O1x, O1y, ON1x, ON1y, s[6], s[7], Q3x, Q3y);
  canon(O2x, O2y, ON2x, ON2y, d[6], d[7], Q4x, Q4y);
  double r = 1.0 / P3y;
  const double P5x = P3x * r, P5y = f1 * r;
  r = 1.0 / P4y;
  const double P6x = P4x * r, P6y = f2 * r;
  r = 1.0 / Q3y;
  const double Q7x = Q3x * r - P5x, Q7y = f1 * r - P5y;
  r = 1.0 / Q4y;
  const double Q8x = Q4x * r - P6x, Q8y = f2 * r - P6y;
  const double sp = (Q8x + Q8y) / (Q7x + Q7y);  // a + b
  const double sm = (Q8x - Q8y) / (Q7x - Q7y);  // a - b
  const double a = (sp + sm) * 0.5, b = (sp - sm) * 0.5;
  const double u = P6x - a * P5x - b * P5y;
  const double v = P6y - b * P5x - a * P5y;
  // K = H_S2^-1 H_K
  const double K[3][3] = {{ON2x * a + O2x * b, ON2x * u - ON2y + O2x * v, ON2x * b + O2x * a},
                          {ON2y * a + O2y * b, ON2y * u + ON2x + O2y * v, ON2y * b + O2y * a},
                          {b, v, a}};
  // H = K H_S1 with H_S1 = [[ON1x, ON1y, tx], [-ON1y, ON1x, ty], [0, 0, f1]]
  const double tx = -(ON1x * O1x + ON1y * O1y);
  const double ty = ON1y * O1x - ON1x * O1y;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    H[3 * i + 0] = K[i][0] * ON1x - K[i][1] * ON1y;
    H[3 * i + 1] = K[i][0] * ON1y + K[i][1] * ON1x;
    H[3 * i + 2] = K[i][0] * tx + K[i][1] * ty + K[i][2] * f1;
  }
  return (quad_side_thin(s) || quad_side_thin(d)) ? kNearDegenerate : 0u;
}

// Simplified SK (Sec. 3.4, eq. SK): the homography up to a similarity from a
// known pattern to one image, Hbar = H_S2^-1 H_K, which maps the pattern's
// canonical frame (anchors at (-1, 0), (1, 0)) to the image. That frame is
// fixed once per pattern, so the pattern's P5 and the reciprocals
// kp = 1 / (Q7.x + Q7.y), km = 1 / (Q7.x - Q7.y) are constants; per image
// only the target-side steps of SKS remain (Table III, second row).
struct SkPattern {
  double P5x, P5y, kp, km;
  uint32_t flags;  // kNearDegenerate if a triangle of the pattern is thin
};

__device__ __forceinline__ uint32_t sk_simplified_solve(const SkPattern &p, const double *d,
                                                        double *H) {
  const double ON2x = (d[2] - d[0]) * 0.5, ON2y = (d[3] - d[1]) * 0.5;
  const double O2x = d[0] + ON2x, O2y = d[1] + ON2y;
  const double f2 = ON2x * ON2x + ON2y * ON2y;
  double dx = d[4] - O2x, dy = d[5] - O2y;
  const double P4x = ON2x * dx + ON2y * dy, P4y = ON2x * dy - ON2y * dx;
  double r = 1.0 / P4y;
  const double P6x = P4x * r, P6y = f2 * r;
  dx = d[6] - O2x;
  dy = d[7] - O2y;
  const double Q4x = ON2x * dx + ON2y * dy, Q4y = ON2x * dy - ON2y * dx;
  r = 1.0 / Q4y;
  const double Q8x = Q4x * r - P6x, Q8y = f2 * r - P6y;
  const double sp = (Q8x + Q8y) * p.kp;  // a + b
  const double sm = (Q8x - Q8y) * p.km;  // a - b
  const double a = (sp + sm) * 0.5, b = (sp - sm) * 0.5;
  const double u = P6x - a * p.P5x - b * p.P5y;
  const double v = P6y - b * p.P5x - a * p.P5y;
  // H_S2^-1 H_K with H_K = [[a, u, b], [0, 1, 0], [b, v, a]]
  H[0] = ON2x * a + O2x * b;
  H[1] = ON2x * u - ON2y + O2x * v;
  H[2] = ON2x * b + O2x * a;
  H[3] = ON2y * a + O2y * b;
  H[4] = ON2y * u + ON2x + O2y * v;
  H[5] = ON2y * b + O2y * a;
  H[6] = b;
  H[7] = v;
  H[8] = a;
  return (p.flags | (quad_side_thin(d) ? kNearDegenerate : 0u));
}

// Affine map through three correspondences M, N, P (Sec. 5.2, eq. AffineACA):
// H_A2^-1 H_A1 (33 operations, third row (0, 0, f_A1)), then its top two rows
// times 1 / f_A1, giving A = [a11 a12 a13; a21 a22 a23] with x' = A (x, y, 1).
// s, d: x_M y_M x_N y_N x_P y_P. Returns the near-degeneracy bit (the triangle
// M N P of either side has height <= kDelta).
__device__ __forceinline__ uint32_t affine_solve(const double *s, const double *d, double *A) {
  const double M1x = s[0], M1y = s[1];
  const double MN1x = s[2] - M1x, MN1y = s[3] - M1y;
  const double MP1x = s[4] - M1x, MP1y = s[5] - M1y;
  const double fA1 = MN1x * MP1y - MN1y * MP1x;
  const double MN2x = d[2] - d[0], MN2y = d[3] - d[1];
  const double MP2x = d[4] - d[0], MP2y = d[5] - d[1];
  const double rows[2][3] = {{MN2x, MP2x, d[0]}, {MN2y, MP2y, d[1]}};
  const double r = 1.0 / fA1;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double h0 = rows[i][0] * MP1y - rows[i][1] * MN1y;
    const double h1 = rows[i][1] * MN1x - rows[i][0] * MP1x;
    const double h2 = rows[i][2] * fA1 - (h0 * M1x + h1 * M1y);
    A[3 * i + 0] = h0 * r;
    A[3 * i + 1] = h1 * r;
    A[3 * i + 2] = h2 * r;
  }
  // triangle heights: A^2 <= delta^2 max(edge^2) on each side
  const double fA2 = MN2x * MP2y - MN2y * MP2x;
  auto thin = [](const double *q, double area) {
    const double e0 = (q[2] - q[0]) * (q[2] - q[0]) + (q[3] - q[1]) * (q[3] - q[1]);
    const double e1 = (q[4] - q[0]) * (q[4] - q[0]) + (q[5] - q[1]) * (q[5] - q[1]);
    const double e2 = (q[4] - q[2]) * (q[4] - q[2]) + (q[5] - q[3]) * (q[5] - q[3]);
    return area * area <= kDelta2 * fmax(fmax(e0, e1), e2);
  };
  return (thin(s, fA1) || thin(d, fA2)) ? kNearDegenerate : 0u;
}

// Scale H by the power of two that brings max|h| into [0.5, 1) (exact) and
// round to float. Zero or non-finite H is written as zeros; returns kZeroH then.
__device__ __forceinline__ uint32_t scale_to_float(const double *H, float *out) {
  double m = 0.0;
  bool bad = false;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double a = fabs(H[i]);
    bad |= !(a <= 1.7976931348623157e308);   // inf or nan
    m = fmax(m, a);
  }
  if (bad || m == 0.0) {
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] = 0.0f;
    return kZeroH;
  }
  int e;
  (void)frexp(m, &e);
#pragma unroll
  for (int i = 0; i < 9; ++i) out[i] = static_cast<float>(ldexp(H[i], -e));
  return 0u;
}

__device__ __forceinline__ bool finite_f(float v) {
  return (__float_as_uint(v) & 0x7f800000u) != 0x7f800000u;
}

// Simplified SK from the float image quadruple to the scaled float Hbar.
__device__ __forceinline__ uint32_t solve_sk(const SkPattern &p, const float *d, float *h) {
  bool fin = true;
#pragma unroll
  for (int k = 0; k < 8; ++k) fin = fin && finite_f(d[k]);
  if (!fin) {
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = 0.0f;
    return kNonfiniteInput | kZeroH;
  }
  double dd[8], H[9];
#pragma unroll
  for (int k = 0; k < 8; ++k) dd[k] = static_cast<double>(d[k]);
  const uint32_t thin = sk_simplified_solve(p, dd, H);
  return thin | scale_to_float(H, h);
}

// Three-point affine from float inputs to the float 2 x 3 map. A non-finite
// result (f_A1 == 0) is written as zeros with kZeroH.
__device__ __forceinline__ uint32_t solve_affine(const float *s, const float *d, float *a) {
  bool fin = true;
#pragma unroll
  for (int k = 0; k < 6; ++k) fin = fin && finite_f(s[k]) && finite_f(d[k]);
  if (!fin) {
#pragma unroll
    for (int i = 0; i < 6; ++i) a[i] = 0.0f;
    return kNonfiniteInput | kZeroH;
  }
  double sd[6], dd[6], A[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    sd[k] = static_cast<double>(s[k]);
    dd[k] = static_cast<double>(d[k]);
  }
  const uint32_t thin = affine_solve(sd, dd, A);
  bool bad = false;
#pragma unroll
  for (int i = 0; i < 6; ++i) bad |= !(fabs(A[i]) <= 1.7976931348623157e308);
#pragma unroll
  for (int i = 0; i < 6; ++i) a[i] = bad ? 0.0f : static_cast<float>(A[i]);
  return thin | (bad ? kZeroH : 0u);
}

// One 4-point problem from float inputs to the scaled float H and its flags.
template <int METHOD>
__device__ __forceinline__ uint32_t solve_quad(const float *s, const float *d, float *h) {
  bool fin = true;
#pragma unroll
  for (int k = 0; k < 8; ++k) fin = fin && finite_f(s[k]) && finite_f(d[k]);
  if (!fin) {
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = 0.0f;
    return kNonfiniteInput | kZeroH;
  }
  double sd[8], dd[8], H[9];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    sd[k] = static_cast<double>(s[k]);
    dd[k] = static_cast<double>(d[k]);
  }
  const uint32_t thin = (METHOD == 0) ? aca_solve(sd, dd, H) : sks_solve(sd, dd, H);
  return thin | scale_to_float(H, h);
}

}  // namespace hg
