"""Reference 4-point homography solvers (oracle; test infrastructure only).

Point order everywhere: M, N, P, Q (ACA anchors M, N, P; fourth point Q; SKS
anchors M, N). A quadruple side is 8 numbers ``xM yM xN yN xP yP xQ yQ``.

Two flavours of every solver:

* ``*_s`` scalar functions written once for any number type that supports
  + - * / (``fractions.Fraction`` for exact rational results, ``float`` for
  FP64, ``oracle.flops.Flop`` for operation counts);
* ``*64`` vectorised NumPy functions over SoA planes of shape (8, n), computed
  in the dtype of the input (float64 for the oracle proper, float32 only to
  emulate a single-precision CPU implementation as context).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

DELTA_PX = 1e-2   # degeneracy threshold on the minimum triangle height (px)


# ---------------------------------------------------------------------------
# helpers

def _half(x):
    """The constant 1/2 in the number type of x."""
    if isinstance(x, Fraction):
        return Fraction(1, 2)
    return 0.5


def _zero(x):
    """0 in the number type of x, produced without arithmetic (so a counting
    type is not charged for it)."""
    if isinstance(x, Fraction):
        return Fraction(0)
    if hasattr(x, "c") and hasattr(x, "v"):
        return type(x)(0.0, x.c)
    return 0.0


def _one(x):
    """1 in the number type of x, produced without arithmetic."""
    if isinstance(x, Fraction):
        return Fraction(1)
    if hasattr(x, "c") and hasattr(x, "v"):
        return type(x)(1.0, x.c)
    return 1.0


def _pts(q):
    return ((q[0], q[1]), (q[2], q[3]), (q[4], q[5]), (q[6], q[7]))


def matmul3(A, B):
    """Plain 3x3 matrix product on nested lists (any number type)."""
    return [[A[i][0] * B[0][j] + A[i][1] * B[1][j] + A[i][2] * B[2][j] for j in range(3)]
            for i in range(3)]


def apply3(H, x, y):
    """Homogeneous image (u, v, w) of (x, y, 1) under H (nested lists)."""
    return (H[0][0] * x + H[0][1] * y + H[0][2],
            H[1][0] * x + H[1][1] * y + H[1][2],
            H[2][0] * x + H[2][1] * y + H[2][2])


# ---------------------------------------------------------------------------
# DLT: the plain definition of the 4-point homography (Sec. 2.1, eqs. for the
# cross-product constraint and the stacked 8x9 system; GPT-LU fixes h33 = 1 and
# solves the 8x8 inhomogeneous system).

def dlt_system(src, dst):
    """Rows of A (8x8) and b (8) with h33 = 1: for each correspondence (x, y) ->
    (u, v): [x, y, 1, 0, 0, 0, -u x, -u y] h = u and
    [0, 0, 0, x, y, 1, -v x, -v y] h = v."""
    A, b = [], []
    for (x, y), (u, v) in zip(_pts(src), _pts(dst)):
        z = _zero(x)
        one = _one(x)
        A.append([x, y, one, z, z, z, -u * x, -u * y])
        b.append(u)
        A.append([z, z, z, x, y, one, -v * x, -v * y])
        b.append(v)
    return A, b


def gauss_solve(A, b):
    """Gaussian elimination with partial pivoting (largest magnitude pivot)."""
    n = len(A)
    M = [list(A[i]) + [b[i]] for i in range(n)]
    for k in range(n):
        p = max(range(k, n), key=lambda i: abs(M[i][k]))
        if M[p][k] == 0:
            raise ZeroDivisionError("singular DLT system")
        M[k], M[p] = M[p], M[k]
        for i in range(k + 1, n):
            f = M[i][k] / M[k][k]
            if f != 0:
                for j in range(k, n + 1):
                    M[i][j] = M[i][j] - f * M[k][j]
    x = [None] * n
    for i in range(n - 1, -1, -1):
        s = M[i][n]
        for j in range(i + 1, n):
            s = s - M[i][j] * x[j]
        x[i] = s / M[i][i]
    return x


def dlt_s(src, dst):
    """Exact (for Fraction input) DLT homography with h33 = 1, nested lists."""
    A, b = dlt_system(src, dst)
    h = gauss_solve(A, b)
    one = _one(h[0])
    return [[h[0], h[1], h[2]], [h[3], h[4], h[5]], [h[6], h[7], one]]


def _normalising_transform(x, y):
    """Hartley normalisation: centroid to the origin, mean distance sqrt(2)."""
    cx, cy = x.mean(axis=0), y.mean(axis=0)
    d = np.sqrt((x - cx) ** 2 + (y - cy) ** 2).mean(axis=0)
    s = np.sqrt(2.0) / d
    n = x.shape[1]
    T = np.zeros((n, 3, 3))
    T[:, 0, 0] = s
    T[:, 1, 1] = s
    T[:, 0, 2] = -s * cx
    T[:, 1, 2] = -s * cy
    T[:, 2, 2] = 1.0
    return T


def dlt64(src, dst):
    """Normalised DLT in float64 over SoA planes (8, n) -> (n, 3, 3).

    Each side is normalised (Hartley), the 8x8 system with h33 = 1 is solved by
    LAPACK's LU with partial pivoting, and the result is denormalised."""
    s = np.asarray(src, np.float64)
    d = np.asarray(dst, np.float64)
    x1, y1, x2, y2 = s[0::2], s[1::2], d[0::2], d[1::2]        # (4, n)
    T1 = _normalising_transform(x1, y1)
    T2 = _normalising_transform(x2, y2)
    n = s.shape[1]
    X1 = T1[:, 0, 0] * x1 + T1[:, 0, 2]
    Y1 = T1[:, 1, 1] * y1 + T1[:, 1, 2]
    X2 = T2[:, 0, 0] * x2 + T2[:, 0, 2]
    Y2 = T2[:, 1, 1] * y2 + T2[:, 1, 2]
    A = np.zeros((n, 8, 8))
    b = np.zeros((n, 8))
    for k in range(4):
        x, y, u, v = X1[k], Y1[k], X2[k], Y2[k]
        r = 2 * k
        A[:, r, 0], A[:, r, 1], A[:, r, 2] = x, y, 1.0
        A[:, r, 6], A[:, r, 7] = -u * x, -u * y
        b[:, r] = u
        A[:, r + 1, 3], A[:, r + 1, 4], A[:, r + 1, 5] = x, y, 1.0
        A[:, r + 1, 6], A[:, r + 1, 7] = -v * x, -v * y
        b[:, r + 1] = v
    h = np.linalg.solve(A, b[..., None])[..., 0]
    Hn = np.concatenate([h, np.ones((n, 1))], axis=1).reshape(n, 3, 3)
    return np.linalg.inv(T2) @ Hn @ T1


# ---------------------------------------------------------------------------
# ACA (Sec. 4.2-4.4): H = H_A2^-1 H_C H_A1.

def aca_s(src, dst):
    """ACA homography up to scale in the structured 85-FLOP order.

    Steps (Table IV): H_A1 from MN1, MP1 and f_A1 (eqs. AffineExpresion,
    f_A_1), likewise H_A2 (7 + 7); the fourth point mapped by the affinities,
    Q3 = H_A1 Q1 and Q4 = H_A2 Q2 (eq. Q3), t1, t2 (eq. t1) and the
    division-free core c11, c22, c33 (eqs. H_C_2, C_11) (28); the composition
    L = H_A2^-1 H_C (10) and H = L H_A1 (33). Returns nested lists."""
    (M1x, M1y), (N1x, N1y), (P1x, P1y), (Q1x, Q1y) = _pts(src)
    (M2x, M2y), (N2x, N2y), (P2x, P2y), (Q2x, Q2y) = _pts(dst)
    # first affine transformation
    MN1x = N1x - M1x
    MN1y = N1y - M1y
    MP1x = P1x - M1x
    MP1y = P1y - M1y
    fA1 = MN1x * MP1y - MN1y * MP1x
    # last affine transformation
    MN2x = N2x - M2x
    MN2y = N2y - M2y
    MP2x = P2x - M2x
    MP2y = P2y - M2y
    fA2 = MN2x * MP2y - MN2y * MP2x
    # core transformation from the fourth correspondence
    MQ1x = Q1x - M1x
    MQ1y = Q1y - M1y
    MQ2x = Q2x - M2x
    MQ2y = Q2y - M2y
    Q3x = MQ1x * MP1y - MQ1y * MP1x
    Q3y = MN1x * MQ1y - MN1y * MQ1x
    Q4x = MQ2x * MP2y - MQ2y * MP2x
    Q4y = MN2x * MQ2y - MN2y * MQ2x
    t1 = fA1 - Q3x - Q3y
    t2 = fA2 - Q4x - Q4y
    c11 = t1 * Q3y * Q4x
    c22 = t1 * Q3x * Q4y
    c33 = t2 * Q3x * Q3y
    d11 = c11 - c33
    d22 = c22 - c33
    # L = H_A2^-1 H_C
    mx = M2x * c33
    my = M2y * c33
    L = [[N2x * c11 - mx, P2x * c22 - mx, mx],
         [N2y * c11 - my, P2y * c22 - my, my],
         [d11, d22, c33]]
    # H = L H_A1 with H_A1 = [[MP1y, -MP1x, .], [-MN1y, MN1x, .], [0, 0, fA1]] T(-M1)
    H = []
    for l0, l1, l2 in L:
        h0 = l0 * MP1y - l1 * MN1y
        h1 = l1 * MN1x - l0 * MP1x
        h2 = l2 * fA1 - (h0 * M1x + h1 * M1y)
        H.append([h0, h1, h2])
    return H


def aca_parts_s(src, dst):
    """The ACA sub-transformations as explicit 3x3 matrices (nested lists):
    (H_A1, H_A2, H_A2^-1 up to scale, H_C) per eqs. AffineExpresion,
    inverseAffineOfA1 and H_C_2."""
    (M1x, M1y), (N1x, N1y), (P1x, P1y), (Q1x, Q1y) = _pts(src)
    (M2x, M2y), (N2x, N2y), (P2x, P2y), (Q2x, Q2y) = _pts(dst)
    z = _zero(M1x)
    one = _one(M1x)

    def affine(Mx, My, Nx, Ny, Px, Py):
        MNx, MNy, MPx, MPy = Nx - Mx, Ny - My, Px - Mx, Py - My
        f = MNx * MPy - MNy * MPx
        A = [[MPy, -MPx, z], [-MNy, MNx, z], [z, z, f]]
        T = [[one, z, -Mx], [z, one, -My], [z, z, one]]
        Ainv = [[MNx, MPx, Mx], [MNy, MPy, My], [z, z, one]]
        return matmul3(A, T), Ainv

    HA1, _ = affine(M1x, M1y, N1x, N1y, P1x, P1y)
    HA2, HA2inv = affine(M2x, M2y, N2x, N2y, P2x, P2y)
    Q3 = apply3(HA1, Q1x, Q1y)
    Q4 = apply3(HA2, Q2x, Q2y)
    t1 = Q3[2] - Q3[0] - Q3[1]
    t2 = Q4[2] - Q4[0] - Q4[1]
    c11 = t1 * Q3[1] * Q4[0]
    c22 = t1 * Q3[0] * Q4[1]
    c33 = t2 * Q3[0] * Q3[1]
    HC = [[c11, z, z], [z, c22, z], [c11 - c33, c22 - c33, c33]]
    return HA1, HA2, HA2inv, HC


def aca_matrix_s(src, dst):
    """ACA as the literal triple product H_A2^-1 H_C H_A1 of explicit matrices."""
    HA1, _, HA2inv, HC = aca_parts_s(src, dst)
    return matmul3(matmul3(HA2inv, HC), HA1)


def aca_poly_s(src, dst, printed=False):
    """Polynomial form of H (Sec. 4.5, eq. H_11): [h11 h21 h31 h12 h22 h32 h13 h23
    h33]^T = M(9x3) [c11 c22 c33]^T with f1, f2 as in eq. f_1.

    The third-column entries of rows h13, h23, h33 are taken as M2.x f3,
    M2.y f3, f3 with f3 = N1.x P1.y - N1.y P1.x (so f1 + f2 + f3 = f_A1): this
    is what the factorisation H = [N2 P2 M2; 1 1 1] diag(c) E H_A1 gives. With
    ``printed=True`` the column uses f_A1 as typeset, which does not reproduce
    the product form (kept to document the discrepancy)."""
    (M1x, M1y), (N1x, N1y), (P1x, P1y), (Q1x, Q1y) = _pts(src)
    (M2x, M2y), (N2x, N2y), (P2x, P2y), (Q2x, Q2y) = _pts(dst)
    MN1x, MN1y, MP1x, MP1y = N1x - M1x, N1y - M1y, P1x - M1x, P1y - M1y
    fA1 = MN1x * MP1y - MN1y * MP1x
    MN2x, MN2y, MP2x, MP2y = N2x - M2x, N2y - M2y, P2x - M2x, P2y - M2y
    fA2 = MN2x * MP2y - MN2y * MP2x
    MQ1x, MQ1y, MQ2x, MQ2y = Q1x - M1x, Q1y - M1y, Q2x - M2x, Q2y - M2y
    Q3x = MQ1x * MP1y - MQ1y * MP1x
    Q3y = MN1x * MQ1y - MN1y * MQ1x
    Q4x = MQ2x * MP2y - MQ2y * MP2x
    Q4y = MN2x * MQ2y - MN2y * MQ2x
    t1 = fA1 - Q3x - Q3y
    t2 = fA2 - Q4x - Q4y
    c = (t1 * Q3y * Q4x, t1 * Q3x * Q4y, t2 * Q3x * Q3y)
    f1 = P1x * M1y - P1y * M1x
    f2 = M1x * N1y - M1y * N1x
    f3 = fA1 if printed else N1x * P1y - N1y * P1x
    one = _one(M1x)
    ay = (P1y - M1y, M1y - N1y, N1y - P1y)
    ax = (M1x - P1x, N1x - M1x, P1x - N1x)
    az = (f1, f2, f3)
    tx = (N2x, P2x, M2x)
    ty = (N2y, P2y, M2y)
    tz = (one, one, one)

    def row(t, a):
        return t[0] * a[0] * c[0] + t[1] * a[1] * c[1] + t[2] * a[2] * c[2]

    h11, h21, h31 = row(tx, ay), row(ty, ay), row(tz, ay)
    h12, h22, h32 = row(tx, ax), row(ty, ax), row(tz, ax)
    h13, h23, h33 = row(tx, az), row(ty, az), row(tz, az)
    return [[h11, h12, h13], [h21, h22, h23], [h31, h32, h33]]


def aca64(src, dst):
    """Vectorised ACA (same structured order as ``aca_s``) over SoA planes
    (8, n); computed in the input dtype. Returns (n, 3, 3)."""
    s = np.asarray(src)
    d = np.asarray(dst)
    H = aca_s(list(s), list(d))
    out = np.empty((s.shape[1], 3, 3), dtype=np.result_type(s, d))
    for i in range(3):
        for j in range(3):
            out[:, i, j] = H[i][j]
    return out


# ---------------------------------------------------------------------------
# SKS (Sec. 3): H = H_S2^-1 H_K H_S1.

def _similarity_s(Mx, My, Nx, Ny):
    """Midpoint O, half-vector ON and f_S (eqs. 3_2_1, 3_2_2, fOfS1)."""
    h = _half(Mx)
    ONx = (Nx - Mx) * h
    ONy = (Ny - My) * h
    Ox = Mx + ONx
    Oy = My + ONy
    f = ONx * ONx + ONy * ONy
    return Ox, Oy, ONx, ONy, f


def _canon_s(Ox, Oy, ONx, ONy, Px, Py):
    """(x, y) of H_S P (homogeneous weight f_S): rotate-scale the offset from O."""
    dx = Px - Ox
    dy = Py - Oy
    return ONx * dx + ONy * dy, ONx * dy - ONy * dx


def sks_s(src, dst):
    """SKS homography (no normalisation) in the order of Table III.

    H_S1, H_S2 map the anchors M, N to (-1, 0), (1, 0) (eq. 3_2_4). P, Q are
    mapped by H_S then by H_E (swap of y and w), giving P5, P6, Q5, Q6 as
    inhomogeneous points; Q7 = Q5 - P5 and Q8 = Q6 - P6 (translations H_T1,
    H_T2). The hyperbolic rotation-scale (a, b) solves eq. 4; summing and
    subtracting its two equations gives a + b and a - b directly. Then u, v
    (kernel parameters) and H = H_S2^-1 H_K H_S1 with H_K of eq. H_K."""
    (M1x, M1y), (N1x, N1y), (P1x, P1y), (Q1x, Q1y) = _pts(src)
    (M2x, M2y), (N2x, N2y), (P2x, P2y), (Q2x, Q2y) = _pts(dst)
    O1x, O1y, ON1x, ON1y, f1 = _similarity_s(M1x, M1y, N1x, N1y)
    O2x, O2y, ON2x, ON2y, f2 = _similarity_s(M2x, M2y, N2x, N2y)
    # P3 = H_S1 P1 (weight f1); P5 = inhomogeneous H_E P3 = (P3.x / P3.y, f1 / P3.y)
    P3x, P3y = _canon_s(O1x, O1y, ON1x, ON1y, P1x, P1y)
    r = 1 / P3y
    P5x, P5y = P3x * r, f1 * r
    P4x, P4y = _canon_s(O2x, O2y, ON2x, ON2y, P2x, P2y)
    r = 1 / P4y
    P6x, P6y = P4x * r, f2 * r
    Q3x, Q3y = _canon_s(O1x, O1y, ON1x, ON1y, Q1x, Q1y)
    r = 1 / Q3y
    Q7x, Q7y = Q3x * r - P5x, f1 * r - P5y
    Q4x, Q4y = _canon_s(O2x, O2y, ON2x, ON2y, Q2x, Q2y)
    r = 1 / Q4y
    Q8x, Q8y = Q4x * r - P6x, f2 * r - P6y
    # eq. 4: Q8 = [[a, b], [b, a]] Q7
    s = (Q8x + Q8y) / (Q7x + Q7y)      # a + b
    d = (Q8x - Q8y) / (Q7x - Q7y)      # a - b
    h = _half(s)
    a = (s + d) * h
    b = (s - d) * h
    u = P6x - a * P5x - b * P5y
    v = P6y - b * P5x - a * P5y
    # K = H_S2^-1 H_K, H_S2^-1 = [[ON2x, -ON2y, O2x], [ON2y, ON2x, O2y], [0, 0, 1]]
    K = [[ON2x * a + O2x * b, ON2x * u - ON2y + O2x * v, ON2x * b + O2x * a],
         [ON2y * a + O2y * b, ON2y * u + ON2x + O2y * v, ON2y * b + O2y * a],
         [b, v, a]]
    # H = K H_S1, H_S1 = [[ON1x, ON1y, tx], [-ON1y, ON1x, ty], [0, 0, f1]]
    tx = -(ON1x * O1x + ON1y * O1y)
    ty = ON1y * O1x - ON1x * O1y
    H = []
    for k0, k1, k2 in K:
        H.append([k0 * ON1x - k1 * ON1y, k0 * ON1y + k1 * ON1x, k0 * tx + k1 * ty + k2 * f1])
    return H


def sks_parts_s(src, dst):
    """SKS sub-transformations as explicit matrices: (H_S1, H_S2, H_S2^-1, H_K)."""
    (M1x, M1y), (N1x, N1y), (P1x, P1y), (Q1x, Q1y) = _pts(src)
    (M2x, M2y), (N2x, N2y), (P2x, P2y), (Q2x, Q2y) = _pts(dst)
    z = _zero(M1x)
    one = _one(M1x)

    def sim(Mx, My, Nx, Ny):
        Ox, Oy, ONx, ONy, f = _similarity_s(Mx, My, Nx, Ny)
        R = [[ONx, ONy, z], [-ONy, ONx, z], [z, z, f]]
        T = [[one, z, -Ox], [z, one, -Oy], [z, z, one]]
        inv = [[ONx, -ONy, Ox], [ONy, ONx, Oy], [z, z, one]]
        return matmul3(R, T), inv

    HS1, _ = sim(M1x, M1y, N1x, N1y)
    HS2, HS2inv = sim(M2x, M2y, N2x, N2y)
    H = sks_s(src, dst)
    # H_K = H_S2 H H_S1^-1 up to scale; rebuild it from the parameters instead
    O1x, O1y, ON1x, ON1y, f1 = _similarity_s(M1x, M1y, N1x, N1y)
    O2x, O2y, ON2x, ON2y, f2 = _similarity_s(M2x, M2y, N2x, N2y)
    P3x, P3y = _canon_s(O1x, O1y, ON1x, ON1y, P1x, P1y)
    P4x, P4y = _canon_s(O2x, O2y, ON2x, ON2y, P2x, P2y)
    Q3x, Q3y = _canon_s(O1x, O1y, ON1x, ON1y, Q1x, Q1y)
    Q4x, Q4y = _canon_s(O2x, O2y, ON2x, ON2y, Q2x, Q2y)
    P5x, P5y = P3x / P3y, f1 / P3y
    P6x, P6y = P4x / P4y, f2 / P4y
    Q7x, Q7y = Q3x / Q3y - P5x, f1 / Q3y - P5y
    Q8x, Q8y = Q4x / Q4y - P6x, f2 / Q4y - P6y
    s = (Q8x + Q8y) / (Q7x + Q7y)
    d = (Q8x - Q8y) / (Q7x - Q7y)
    a = (s + d) * _half(s)
    b = (s - d) * _half(s)
    u = P6x - a * P5x - b * P5y
    v = P6y - b * P5x - a * P5y
    HK = [[a, u, b], [z, one, z], [b, v, a]]
    return HS1, HS2, HS2inv, HK, H


def sks64(src, dst):
    """Vectorised SKS over SoA planes (8, n), computed in the input dtype."""
    s = np.asarray(src)
    d = np.asarray(dst)
    with np.errstate(divide="ignore", invalid="ignore"):
        H = sks_s(list(s), list(d))
    out = np.empty((s.shape[1], 3, 3), dtype=np.result_type(s, d))
    for i in range(3):
        for j in range(3):
            out[:, i, j] = H[i][j]
    return out


# ---------------------------------------------------------------------------
# Simplified SK (Sec. 3.4, eq. SK): homography up to a similarity between a
# known object pattern and its images. The object's anchors M, N fix a
# canonical frame once per pattern (H_S1 is then never formed per problem), so
# P5, Q5 and Q7 of the pattern are constants and each image only pays for
# H_S2, P6, Q8, the kernel parameters and H_S2^-1 H_K (Table III, second row).

def sk_pattern_s(obj):
    """Per-pattern constants of the simplified SK for the object points
    ``obj`` = M N P Q (8 numbers, object coordinates).

    Returns (P5x, P5y, kp, km, HS1): P5 is the pattern's P after H_S1 and the
    swap H_E, kp = 1 / (Q7.x + Q7.y) and km = 1 / (Q7.x - Q7.y) with
    Q7 = Q5 - P5 (the denominators of the (a, b) solve), and HS1 is the
    similarity of eq. 3_2_4 as a matrix, so that the complete homography is
    H = Hbar H_S1 up to scale."""
    (M1x, M1y), (N1x, N1y), (P1x, P1y), (Q1x, Q1y) = _pts(obj)
    O1x, O1y, ON1x, ON1y, f1 = _similarity_s(M1x, M1y, N1x, N1y)
    P3x, P3y = _canon_s(O1x, O1y, ON1x, ON1y, P1x, P1y)
    r = 1 / P3y
    P5x, P5y = P3x * r, f1 * r
    Q3x, Q3y = _canon_s(O1x, O1y, ON1x, ON1y, Q1x, Q1y)
    r = 1 / Q3y
    Q7x, Q7y = Q3x * r - P5x, f1 * r - P5y
    kp = 1 / (Q7x + Q7y)
    km = 1 / (Q7x - Q7y)
    z = _zero(M1x)
    tx = -(ON1x * O1x + ON1y * O1y)
    ty = ON1y * O1x - ON1x * O1y
    HS1 = [[ON1x, ON1y, tx], [-ON1y, ON1x, ty], [z, z, f1]]
    return P5x, P5y, kp, km, HS1


def sk_simplified_s(pattern, dst):
    """Hbar = H_S2^-1 H_K (eq. SK) for one image ``dst`` = M2 N2 P2 Q2 of the
    pattern whose constants ``pattern`` come from ``sk_pattern_s``; Hbar maps
    the pattern's canonical frame to the image. The steps are those of SKS on
    the target side; the (a, b) solve multiplies by the pattern's reciprocals
    kp, km instead of dividing."""
    P5x, P5y, kp, km = pattern[:4]
    (M2x, M2y), (N2x, N2y), (P2x, P2y), (Q2x, Q2y) = _pts(dst)
    O2x, O2y, ON2x, ON2y, f2 = _similarity_s(M2x, M2y, N2x, N2y)
    P4x, P4y = _canon_s(O2x, O2y, ON2x, ON2y, P2x, P2y)
    r = 1 / P4y
    P6x, P6y = P4x * r, f2 * r
    Q4x, Q4y = _canon_s(O2x, O2y, ON2x, ON2y, Q2x, Q2y)
    r = 1 / Q4y
    Q8x, Q8y = Q4x * r - P6x, f2 * r - P6y
    s = (Q8x + Q8y) * kp       # a + b
    d = (Q8x - Q8y) * km       # a - b
    h = _half(s)
    a = (s + d) * h
    b = (s - d) * h
    u = P6x - a * P5x - b * P5y
    v = P6y - b * P5x - a * P5y
    return [[ON2x * a + O2x * b, ON2x * u - ON2y + O2x * v, ON2x * b + O2x * a],
            [ON2y * a + O2y * b, ON2y * u + ON2x + O2y * v, ON2y * b + O2y * a],
            [b, v, a]]


def sk64(obj, dst):
    """Vectorised simplified SK: one pattern ``obj`` (8 floats) and SoA target
    planes (8, n) in float64. Returns (Hbar (n, 3, 3), H_S1 (3, 3))."""
    pat = sk_pattern_s([float(v) for v in obj])
    d = np.asarray(dst, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        H = sk_simplified_s(pat, list(d))
    out = np.empty((d.shape[1], 3, 3))
    for i in range(3):
        for j in range(3):
            out[:, i, j] = H[i][j]
    return out, np.array(pat[4], dtype=np.float64)


# ---------------------------------------------------------------------------
# Rectangle source (Sec. 5.3, eqs. H_A1_square .. H_square; Algorithm 1).

def aca_rect_s(x0, y0, w, r, dst, square=False):
    """Algorithm 1: homography from the rectangle with upper-left vertex
    (x0, y0), width w and aspect ratio r (width / height) to the target corners
    ``dst`` = M2 N2 P2 Q2 (M = top-left, N = top-right, Q = bottom-right,
    P = bottom-left). Vectors are handled elementwise; multiplications by the
    homogeneous coordinate 1 are not performed, and with ``square=True`` the
    multiplication by r = 1 is skipped. Returns H as nested lists."""
    (M2x, M2y), (N2x, N2y), (P2x, P2y), (Q2x, Q2y) = _pts(dst)
    # step 1: difference vectors
    d1 = (N2x - M2x, P2x - M2x, Q2x - M2x)
    d2 = (N2y - M2y, P2y - M2y, Q2y - M2y)
    # step 2: cross product c = d1 x d2
    c0 = d1[1] * d2[2] - d1[2] * d2[1]
    c1 = d1[2] * d2[0] - d1[0] * d2[2]
    c2 = d1[0] * d2[1] - d1[1] * d2[0]
    # step 3: b = Sum(c) m2
    S = c0 + c1 + c2
    b = (S * M2x, S * M2y, S)
    # step 4: first two columns
    h1 = (c0 * N2x - b[0], c0 * N2y - b[1], c0 - b[2])
    h2 = (c1 * P2x - b[0], c1 * P2y - b[1], c1 - b[2])
    if not square:
        h2 = (r * h2[0], r * h2[1], r * h2[2])
    # step 5: last column
    h3 = tuple(w * b[i] - x0 * h1[i] - y0 * h2[i] for i in range(3))
    return [[h1[0], h2[0], h3[0]], [h1[1], h2[1], h3[1]], [h1[2], h2[2], h3[2]]]


def rect_corners(x0, y0, w, r):
    """Source quadruple (M N P Q) of a rectangle: TL, TR, BL, BR."""
    hgt = w / r
    return [x0, y0, x0 + w, y0, x0, y0 + hgt, x0 + w, y0 + hgt]


def aca_rect64(x0, y0, w, r, dst, square=False):
    """Vectorised Algorithm 1 over target planes (8, n); (n, 3, 3)."""
    d = np.asarray(dst)
    H = aca_rect_s(x0, y0, w, r, list(d), square=square)
    out = np.empty((d.shape[1], 3, 3), dtype=d.dtype)
    for i in range(3):
        for j in range(3):
            out[:, i, j] = H[i][j]
    return out


# ---------------------------------------------------------------------------
# Affine case (Sec. 5.2, eq. AffineACA): H_C = I, H_A = H_A2^-1 H_A1.

def affine_aca_s(src3, dst3):
    """Affine map through three correspondences (M, N, P) as H_A2^-1 H_A1
    (33 FLOPs, up to the scale f_A1). ``src3``/``dst3`` hold 6 numbers."""
    (M1x, M1y), (N1x, N1y), (P1x, P1y) = (src3[0], src3[1]), (src3[2], src3[3]), (src3[4], src3[5])
    (M2x, M2y), (N2x, N2y), (P2x, P2y) = (dst3[0], dst3[1]), (dst3[2], dst3[3]), (dst3[4], dst3[5])
    MN1x, MN1y, MP1x, MP1y = N1x - M1x, N1y - M1y, P1x - M1x, P1y - M1y
    fA1 = MN1x * MP1y - MN1y * MP1x
    MN2x, MN2y, MP2x, MP2y = N2x - M2x, N2y - M2y, P2x - M2x, P2y - M2y
    H = []
    for a, b, m in ((MN2x, MP2x, M2x), (MN2y, MP2y, M2y)):
        h0 = a * MP1y - b * MN1y
        h1 = b * MN1x - a * MP1x
        h2 = m * fA1 - (h0 * M1x + h1 * M1y)
        H.append([h0, h1, h2])
    z = _zero(M1x)
    H.append([z, z, fA1])
    return H


def affine_normalised_s(src3, dst3):
    """The affine map of ``affine_aca_s`` with its third row brought to
    (0, 0, 1): the top two rows multiplied by 1 / f_A1 (one division and six
    multiplications). Returns the 2 x 3 matrix [A | t] with x' = A x + t."""
    H = affine_aca_s(src3, dst3)
    r = 1 / H[2][2]
    return [[H[0][0] * r, H[0][1] * r, H[0][2] * r], [H[1][0] * r, H[1][1] * r, H[1][2] * r]]


def affine64(src, dst):
    """Vectorised normalised affine over SoA planes (6, n) in float64;
    returns (n, 2, 3) (inf or nan where f_A1 = 0)."""
    s = np.asarray(src, np.float64)
    d = np.asarray(dst, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        A = affine_normalised_s(list(s), list(d))
    out = np.empty((s.shape[1], 2, 3))
    for i in range(2):
        for j in range(3):
            out[:, i, j] = A[i][j]
    return out


# ---------------------------------------------------------------------------
# Degeneracy flag, scaling, comparison (conventions of this implementation;
# the paper defines H only up to scale and has no degeneracy handling).

FLAG_NEAR_DEGENERATE = 1   # minimum triangle height <= delta on either side
FLAG_NONFINITE_INPUT = 2   # some input coordinate is inf or nan
FLAG_ZERO_H = 4            # H is zero or non-finite; written as all zeros

_EDGES = {"MN": (0, 1), "MP": (0, 2), "MQ": (0, 3), "NP": (1, 2), "NQ": (1, 3), "PQ": (2, 3)}
# triangles as (vertices, edges); their doubled areas are f_A, Q.x, Q.y and t
_TRIS = (("MNP", ("MN", "MP", "NP")), ("MQP", ("MQ", "MP", "PQ")),
         ("MNQ", ("MN", "MQ", "NQ")), ("NPQ", ("NP", "NQ", "PQ")))


def side_heights(q):
    """Minimum height of each of the 4 triangles of one side (planes (8, n),
    float64): doubled area divided by the longest edge."""
    q = np.asarray(q, np.float64)
    X, Y = q[0::2], q[1::2]

    def cross(a, b, c):
        return (X[b] - X[a]) * (Y[c] - Y[a]) - (Y[b] - Y[a]) * (X[c] - X[a])

    L2 = {k: (X[j] - X[i]) ** 2 + (Y[j] - Y[i]) ** 2 for k, (i, j) in _EDGES.items()}
    idx = {"M": 0, "N": 1, "P": 2, "Q": 3}
    out = []
    for name, edges in _TRIS:
        a, b, c = (idx[ch] for ch in name)
        A = np.abs(cross(a, b, c))
        Lm = np.maximum(np.maximum(L2[edges[0]], L2[edges[1]]), L2[edges[2]])
        with np.errstate(divide="ignore", invalid="ignore"):
            out.append(np.where(Lm > 0, A / np.sqrt(Lm), 0.0))
    return np.stack(out)


def min_height(src, dst):
    """Smallest triangle height over the 8 triangles of a quadruple pair."""
    return np.minimum(side_heights(src).min(axis=0), side_heights(dst).min(axis=0))


def degeneracy_flags(src, dst, delta=DELTA_PX):
    """Flag bits per quadruple: bit0 iff the minimum triangle height over the
    four triangles of each side is <= delta px, bit1 iff an input is not
    finite."""
    s = np.asarray(src, np.float64)
    d = np.asarray(dst, np.float64)
    fin = np.isfinite(s).all(axis=0) & np.isfinite(d).all(axis=0)
    with np.errstate(invalid="ignore"):
        near = min_height(s, d) <= delta
    return (np.where(near & fin, FLAG_NEAR_DEGENERATE, 0)
            | np.where(fin, 0, FLAG_NONFINITE_INPUT)).astype(np.uint8)


def triangle_heights(t):
    """Height of the triangle M N P over its longest edge for planes (6, n)
    ``xM yM xN yN xP yP`` (float64)."""
    t = np.asarray(t, np.float64)
    X, Y = t[0::2], t[1::2]
    A = np.abs((X[1] - X[0]) * (Y[2] - Y[0]) - (Y[1] - Y[0]) * (X[2] - X[0]))
    L2 = [(X[j] - X[i]) ** 2 + (Y[j] - Y[i]) ** 2 for i, j in ((0, 1), (0, 2), (1, 2))]
    Lm = np.maximum(np.maximum(L2[0], L2[1]), L2[2])
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(Lm > 0, A / np.sqrt(Lm), 0.0)


def affine_flags(src, dst, delta=DELTA_PX):
    """Flag bits of the 3-point affine problem: bit0 iff the triangle M N P of
    either side has height <= delta, bit1 iff an input is not finite."""
    s = np.asarray(src, np.float64)
    d = np.asarray(dst, np.float64)
    fin = np.isfinite(s).all(axis=0) & np.isfinite(d).all(axis=0)
    with np.errstate(invalid="ignore"):
        near = np.minimum(triangle_heights(s), triangle_heights(d)) <= delta
    return (np.where(near & fin, FLAG_NEAR_DEGENERATE, 0)
            | np.where(fin, 0, FLAG_NONFINITE_INPUT)).astype(np.uint8)


def sk_flags(obj, dst, delta=DELTA_PX):
    """Flag bits of the simplified SK: bit0 iff a triangle of the pattern
    ``obj`` (8 numbers) or of the image quadruple has height <= delta, bit1
    iff an image coordinate is not finite."""
    d = np.asarray(dst, np.float64)
    pat_thin = bool(side_heights(np.asarray(obj, np.float64)[:, None]).min() <= delta)
    fin = np.isfinite(d).all(axis=0)
    with np.errstate(invalid="ignore"):
        near = (side_heights(d).min(axis=0) <= delta) | pat_thin
    return (np.where(near & fin, FLAG_NEAR_DEGENERATE, 0)
            | np.where(fin, 0, FLAG_NONFINITE_INPUT)).astype(np.uint8)


def pow2_f32(H):
    """Scale each H (..., 3, 3) by the power of two that brings its largest
    magnitude into [0.5, 1) (exact), then round to float32. Zero or non-finite
    H become all zeros; returns (H32, ok)."""
    H = np.asarray(H, np.float64)
    m = np.abs(H).max(axis=(-2, -1))
    ok = np.isfinite(m) & (m > 0)
    e = np.frexp(np.where(ok, m, 1.0))[1]
    Hs = np.ldexp(np.where(ok[..., None, None], H, 0.0), -e[..., None, None])
    return Hs.astype(np.float32), ok


def normalise(H):
    """Frobenius-normalised H (..., 3, 3) in float64."""
    H = np.asarray(H, np.float64)
    return H / np.linalg.norm(H.reshape(H.shape[:-2] + (9,)), axis=-1)[..., None, None]


def herr(A, B):
    """Distance between homographies up to scale: both Frobenius-normalised, the
    sign of A chosen to agree with B, then the Frobenius norm of the
    difference."""
    a = normalise(A).reshape(-1, 9)
    b = normalise(B).reshape(-1, 9)
    sgn = np.where((a * b).sum(axis=1) < 0, -1.0, 1.0)
    return np.linalg.norm(a * sgn[:, None] - b, axis=1).reshape(np.shape(A)[:-2])


def exact_h(src_row, dst_row, solver=None):
    """Exact rational homography (h33 = 1) of one quadruple given as float
    sequences of length 8; ``solver`` defaults to the DLT definition."""
    s = [Fraction(float(v)) for v in src_row]
    d = [Fraction(float(v)) for v in dst_row]
    H = (solver or dlt_s)(s, d)
    k = H[2][2]
    return np.array([[float(x / k) for x in r] for r in H])
