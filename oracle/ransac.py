"""RANSAC hypothesise-and-verify reference (oracle; test infrastructure only).

What is computed (the paper's RANSAC stage: sample 4 correspondences, solve the
4-point homography, verify inliers, keep the best hypothesis):

* hypothesis j draws 4 distinct indices (``oracle.sampling``) and solves ACA in
  float64 on those correspondences; the result is scaled by a power of two and
  rounded to float32, which is the H that is scored and returned;
* a hypothesis whose sample is degenerate (flag bit set) or whose H is zero has
  count 0 and never wins;
* point i is an inlier of H iff its one-way transfer error
  ``|| pi(H x1_i) - x2_i ||_2`` is at most tau (inclusive); a point mapped to
  infinity (w = 0) is an outlier;
* best = the largest count, ties to the lowest hypothesis index; the mask marks
  the inliers of the best H (no refit); with no valid hypothesis best = -1.

The verification here is evaluated in float64 with a division and a square
root, i.e. by the definition. Counts are compared exactly except for points
whose transfer error lies within ``band_px`` (1e-4 px) of the threshold, where
any two correct evaluations may disagree (``count_lo`` / ``count_hi``).
``decision_band`` is a diagnostic: it bounds how far a float32 division-free
evaluation of the same test may stray, i.e. how wide the exemption would have
to be for a scorer that decides in float32 alone.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np

from . import homography as hg
from .sampling import sample_indices

U32 = 2.0 ** -24   # unit roundoff of float32


def hypotheses(corr, n_hyp, seed, pair=0):
    """Sample and solve: returns (idx (4, n_hyp), H32 (n_hyp, 3, 3) float32,
    flags (n_hyp,) uint8, valid (n_hyp,) bool)."""
    corr = np.asarray(corr, np.float32)
    n = corr.shape[1]
    idx = sample_indices(n, n_hyp, seed, pair)
    src = np.empty((8, n_hyp), np.float32)
    dst = np.empty((8, n_hyp), np.float32)
    for k in range(4):
        src[2 * k] = corr[0, idx[k]]
        src[2 * k + 1] = corr[1, idx[k]]
        dst[2 * k] = corr[2, idx[k]]
        dst[2 * k + 1] = corr[3, idx[k]]
    H64 = hg.aca64(src.astype(np.float64), dst.astype(np.float64))
    flags = hg.degeneracy_flags(src, dst)
    H32, ok = hg.pow2_f32(H64)
    flags = flags | np.where(ok, 0, hg.FLAG_ZERO_H).astype(np.uint8)
    H32[flags != 0] = 0.0
    return idx, H32, flags, flags == 0


def transfer_error(H, corr):
    """One-way transfer error (n_h, n_pts) in float64 for H (n_h, 3, 3)."""
    H = np.asarray(H, np.float64)
    x1, y1, x2, y2 = (np.asarray(c, np.float64) for c in corr)
    u = H[:, 0, 0, None] * x1 + H[:, 0, 1, None] * y1 + H[:, 0, 2, None]
    v = H[:, 1, 0, None] * x1 + H[:, 1, 1, None] * y1 + H[:, 1, 2, None]
    w = H[:, 2, 0, None] * x1 + H[:, 2, 1, None] * y1 + H[:, 2, 2, None]
    with np.errstate(divide="ignore", invalid="ignore"):
        d = np.hypot(u / w - x2, v / w - y2)
    return np.where(w == 0, np.inf, d)


def decision_band(H, corr, tau):
    """Per (hypothesis, point) bound, in px of transfer error, on how far a
    float32 evaluation of the division-free inlier test can move the decision.

    The evaluation bounded here: with c = 1/tau rounded to float, rows 1-2 of
    H and the target point are multiplied by c (each product rounded), then
    u', v', w from 3-term dot products, ru' = u' - (c x2) w, rv' likewise, and
    inlier iff ru'^2 + rv'^2 <= w^2 -- in exact arithmetic the same test as
    ||pi(H x1) - x2|| <= tau. The H entries may also be one float32 ulp off.

    Each 3-term dot product (two fused or separate roundings, one-ulp
    perturbation of every H entry, the rounding of c h) errs by at most 4u
    times the sum of the magnitudes of its terms (u = 2^-24); the residual
    adds one rounding and the rounding of c x2 (u |x2 w| each). Propagating to
    e = ru^2 + rv^2 - tau^2 w^2 (three more roundings on each square) bounds
    the error of e; since e = w^2 (dist - tau)(dist + tau), the decision can
    only flip if |dist - tau| <= |error of e| / (w^2 (dist + tau)). The
    rounding of c moves the effective threshold by at most 2u tau. The sum is
    returned, doubled for safety."""
    Hs = np.asarray(H, np.float64)
    H = np.abs(Hs)
    x1, y1, x2, y2 = (np.asarray(c, np.float64) for c in corr)
    ax1, ay1, ax2, ay2 = np.abs(x1), np.abs(y1), np.abs(x2), np.abs(y2)
    Su = H[:, 0, 0, None] * ax1 + H[:, 0, 1, None] * ay1 + H[:, 0, 2, None]
    Sv = H[:, 1, 0, None] * ax1 + H[:, 1, 1, None] * ay1 + H[:, 1, 2, None]
    Sw = H[:, 2, 0, None] * ax1 + H[:, 2, 1, None] * ay1 + H[:, 2, 2, None]
    u = Hs[:, 0, 0, None] * x1 + Hs[:, 0, 1, None] * y1 + Hs[:, 0, 2, None]
    v = Hs[:, 1, 0, None] * x1 + Hs[:, 1, 1, None] * y1 + Hs[:, 1, 2, None]
    w = Hs[:, 2, 0, None] * x1 + Hs[:, 2, 1, None] * y1 + Hs[:, 2, 2, None]
    ru = u - x2 * w
    rv = v - y2 * w
    Ew = 4 * U32 * Sw
    Eru = 4 * U32 * Su + ax2 * Ew + U32 * (np.abs(u) + 2 * ax2 * np.abs(w))
    Erv = 4 * U32 * Sv + ay2 * Ew + U32 * (np.abs(v) + 2 * ay2 * np.abs(w))
    d = ru * ru + rv * rv
    t = tau * tau * w * w
    Ee = (2 * np.abs(ru) * Eru + Eru ** 2 + 2 * np.abs(rv) * Erv + Erv ** 2 + 3 * U32 * d
          + tau * tau * (2 * np.abs(w) * Ew + Ew ** 2) + 3 * U32 * t)
    with np.errstate(divide="ignore", invalid="ignore"):
        dist = np.sqrt(d) / np.abs(w)
        band = 2.0 * (Ee / (w * w * (dist + tau)) + 2 * U32 * tau)
    return np.where(w == 0, np.inf, band)


def ransac_ref(corr, n_hyp, tau, seed, pair=0, band_px=1e-4, chunk=512):
    """Full single-pair reference. Returns a dict with idx, H32, flags, valid,
    counts (int64, 0 for invalid), count_lo / count_hi (counts with every point
    whose transfer error is within band_px of tau taken as outlier / inlier),
    n_exempt (per hypothesis, the number of such points), best_hyp,
    best_count, best_H (float32), mask (uint8) and mask_exempt (bool: mask
    entries within band_px of tau)."""
    corr = np.asarray(corr, np.float32)
    idx, H32, flags, valid = hypotheses(corr, n_hyp, seed, pair)
    counts = np.zeros(n_hyp, np.int64)
    lo = np.zeros(n_hyp, np.int64)
    hi = np.zeros(n_hyp, np.int64)
    for a in range(0, n_hyp, chunk):
        b = min(n_hyp, a + chunk)
        d = transfer_error(H32[a:b], corr)
        inl = d <= tau
        ex = np.abs(d - tau) < band_px
        v = valid[a:b, None]
        counts[a:b] = (inl & v).sum(axis=1)
        lo[a:b] = (inl & ~ex & v).sum(axis=1)
        hi[a:b] = ((inl | ex) & v).sum(axis=1)
    out = dict(idx=idx, H32=H32, flags=flags, valid=valid, counts=counts,
               count_lo=lo, count_hi=hi, n_exempt=hi - lo)
    if valid.any():
        c = np.where(valid, counts, -1)
        best = int(np.argmax(c))            # first maximum = lowest index
        d = transfer_error(H32[best:best + 1], corr)[0]
        out.update(best_hyp=best, best_count=int(counts[best]), best_H=H32[best].copy(),
                   mask=(d <= tau).astype(np.uint8), mask_exempt=np.abs(d - tau) < band_px)
    else:
        n = corr.shape[1]
        out.update(best_hyp=-1, best_count=0, best_H=np.zeros((3, 3), np.float32),
                   mask=np.zeros(n, np.uint8), mask_exempt=np.zeros(n, bool))
    return out


def brute_force_counts(corr, tau):
    """Inlier count of every 4-subset (by index tuple) of a tiny set, with H
    from the exact DLT definition and the float64 transfer error."""
    corr = np.asarray(corr, np.float64)
    n = corr.shape[1]
    res = {}
    for sub in combinations(range(n), 4):
        src = [v for k in sub for v in (corr[0, k], corr[1, k])]
        dst = [v for k in sub for v in (corr[2, k], corr[3, k])]
        try:
            H = hg.exact_h(src, dst)
        except ZeroDivisionError:
            continue
        res[sub] = int((transfer_error(H[None], corr)[0] <= tau).sum())
    return res


# ---------------------------------------------------------------------------
# Adaptive termination (the RANSAC loop rule of the experiments: as many
# iterations as give, with probability `conf`, at least one all-inlier sample
# for the best inlier ratio found so far, capped at a maximum).

def required_iterations(eps, conf=0.99):
    """k = ceil(log(1 - conf) / log(1 - eps^4)): iterations needed for an
    all-inlier 4-sample with probability conf at inlier ratio eps."""
    import math
    if eps >= 1.0:
        return 1
    if eps <= 0.0:
        return math.inf
    return math.ceil(math.log(1.0 - conf) / math.log1p(-eps ** 4))


def stopping_point(valid, counts, n, n_hyp_max, conf=0.99, round_size=64):
    """Hypotheses evaluated by the sequential adaptive loop: rounds of
    ``round_size`` in index order; after each round eps = best count so far / n,
    and the loop ends once the number evaluated m reaches
    min(required_iterations(eps), n_hyp_max)."""
    m = 0
    for r in range((n_hyp_max + round_size - 1) // round_size):
        m = min((r + 1) * round_size, n_hyp_max)
        c = np.where(valid[:m], counts[:m], -1)
        best_count = int(c.max()) if valid[:m].any() else 0
        if m >= min(required_iterations(best_count / n, conf), n_hyp_max):
            break
    return m


def ransac_adaptive_ref(corr, n_hyp_max, tau, seed, pair=0, conf=0.99, round_size=64,
                        band_px=1e-4, full=None):
    """Adaptive single-pair reference. Hypotheses are evaluated in rounds of
    ``round_size`` (in index order); after each round the best so far gives
    eps = best_count / N, and the loop stops once the number evaluated m
    reaches min(required_iterations(eps), n_hyp_max). Returns the ransac_ref
    dict restricted to the evaluated prefix plus n_eval, and n_eval_min /
    n_eval_max: the stopping points when every exempt point is taken as an
    inlier / an outlier. ``full``: the fixed-count reference of the same pair,
    n_hyp_max, seed and band (ransac_ref), if already computed."""
    if full is None:
        full = ransac_ref(corr, n_hyp_max, tau, seed, pair=pair, band_px=band_px)
    n = np.asarray(corr).shape[1]
    valid, counts = full["valid"], full["counts"]
    m = stopping_point(valid, counts, n, n_hyp_max, conf, round_size)
    out = dict(full)
    out["n_eval"] = m
    # the rule stops no later when counts are larger: bounds on the stopping
    # point over every choice of the exempt points' decisions
    out["n_eval_min"] = stopping_point(valid, full["count_hi"], n, n_hyp_max, conf, round_size)
    out["n_eval_max"] = stopping_point(valid, full["count_lo"], n, n_hyp_max, conf, round_size)
    v = valid[:m]
    if v.any():
        c = np.where(v, counts[:m], -1)
        best = int(np.argmax(c))
        d = transfer_error(full["H32"][best:best + 1], corr)[0]
        out.update(best_hyp=best, best_count=int(counts[best]), best_H=full["H32"][best].copy(),
                   mask=(d <= tau).astype(np.uint8), mask_exempt=np.abs(d - tau) < band_px)
    else:
        out.update(best_hyp=-1, best_count=0, best_H=np.zeros((3, 3), np.float32),
                   mask=np.zeros(n, np.uint8), mask_exempt=np.zeros(n, bool))
    return out
