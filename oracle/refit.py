"""n-point homography refit on RANSAC inliers (oracle; test infrastructure only).

The paper recommends the HO-SVD method (Harker and O'Leary) for n-point
homographies (Sec. 3.5 and the related-work comparison): the DLT system
A h = 0 with rows

    [x y 1 0 0 0 -u x -u y -u]    and    [0 0 0 x y 1 -v x -v y -v]

is reduced to the three unknowns of the last row h3 of H by eliminating the
first two rows in the least-squares sense. With X = [x y 1] (n x 3), D_u =
diag(u), D_v = diag(v) and P the orthogonal projector onto the columns of X:

    h1 = (X^T X)^-1 X^T D_u X h3,   h2 = (X^T X)^-1 X^T D_v X h3,
    M  = [(I - P) D_u X ; (I - P) D_v X]        (2n x 3),
    h3 = the right singular vector of M for its smallest singular value.

Readings of this implementation (the paper gives HO-SVD by reference only):
both point sets are first normalised about their centroids by an isotropic
scale that makes the root-mean-square distance sqrt(2); H maps the source
points (x1, y1) to the targets (x2, y2); the result is denormalised as
T2^-1 Hn T1. Fewer than 4 points give no homography.

Everything is float64 NumPy; P is applied through a QR factorisation of X.
"""
from __future__ import annotations

import numpy as np


def normalisation(x, y):
    """Centroid (cx, cy) and scale s with RMS distance sqrt(2) after
    (x - cx) * s, (y - cy) * s."""
    cx, cy = x.mean(), y.mean()
    ms = ((x - cx) ** 2 + (y - cy) ** 2).mean()
    s = np.sqrt(2.0 / ms)
    return cx, cy, s


def ho_svd(x1, y1, x2, y2):
    """HO-SVD homography (3, 3) from n >= 4 correspondences (float64 arrays);
    returns None when n < 4."""
    x1, y1, x2, y2 = (np.asarray(a, np.float64) for a in (x1, y1, x2, y2))
    n = x1.size
    if n < 4:
        return None
    c1x, c1y, s1 = normalisation(x1, y1)
    c2x, c2y, s2 = normalisation(x2, y2)
    x, y = (x1 - c1x) * s1, (y1 - c1y) * s1
    u, v = (x2 - c2x) * s2, (y2 - c2y) * s2
    X = np.stack([x, y, np.ones(n)], axis=1)
    Q, R = np.linalg.qr(X)

    def resid(Z):                      # (I - P) Z
        return Z - Q @ (Q.T @ Z)

    Mu = resid(u[:, None] * X)
    Mv = resid(v[:, None] * X)
    M = np.concatenate([Mu, Mv], axis=0)
    h3 = np.linalg.svd(M)[2][-1]
    h1 = np.linalg.solve(R, Q.T @ ((u[:, None] * X) @ h3))
    h2 = np.linalg.solve(R, Q.T @ ((v[:, None] * X) @ h3))
    Hn = np.stack([h1, h2, h3])
    T1 = np.array([[s1, 0.0, -s1 * c1x], [0.0, s1, -s1 * c1y], [0.0, 0.0, 1.0]])
    T2inv = np.array([[1.0 / s2, 0.0, c2x], [0.0, 1.0 / s2, c2y], [0.0, 0.0, 1.0]])
    return T2inv @ Hn @ T1


def refit_ref(corr, off, mask):
    """Per pair p (points [off[p], off[p+1]) of the planes corr = x1 y1 x2 y2),
    HO-SVD over the points whose mask byte is non-zero. Returns (H (P, 3, 3)
    float64, zero where fewer than 4 points; n_used (P,) int)."""
    corr = np.asarray(corr, np.float64)
    P = len(off) - 1
    H = np.zeros((P, 3, 3))
    used = np.zeros(P, np.int64)
    for p in range(P):
        a, b = int(off[p]), int(off[p + 1])
        sel = np.nonzero(np.asarray(mask[a:b]))[0] + a
        used[p] = sel.size
        h = ho_svd(corr[0, sel], corr[1, sel], corr[2, sel], corr[3, sel])
        if h is not None:
            H[p] = h
    return H, used


def algebraic_residual(H, x1, y1, x2, y2):
    """The HO objective at H, in the normalised coordinates of the data:
    ||A_n vec(Hn)|| / ||h3_n|| with Hn = T2 H T1^-1 (the quantity HO-SVD
    minimises)."""
    x1, y1, x2, y2 = (np.asarray(a, np.float64) for a in (x1, y1, x2, y2))
    c1x, c1y, s1 = normalisation(x1, y1)
    c2x, c2y, s2 = normalisation(x2, y2)
    T1inv = np.array([[1.0 / s1, 0.0, c1x], [0.0, 1.0 / s1, c1y], [0.0, 0.0, 1.0]])
    T2 = np.array([[s2, 0.0, -s2 * c2x], [0.0, s2, -s2 * c2y], [0.0, 0.0, 1.0]])
    Hn = T2 @ H @ T1inv
    x, y = (x1 - c1x) * s1, (y1 - c1y) * s1
    u, v = (x2 - c2x) * s2, (y2 - c2y) * s2
    X = np.stack([x, y, np.ones(x.size)], axis=1)
    ru = X @ Hn[0] - u * (X @ Hn[2])
    rv = X @ Hn[1] - v * (X @ Hn[2])
    return np.sqrt((ru ** 2).sum() + (rv ** 2).sum()) / np.linalg.norm(Hn[2])
