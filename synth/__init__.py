"""Seeded synthetic workloads for the 4-point homography hot path.

This module only draws random inputs. It holds none of the solver, scoring or
warping arithmetic; the oracle and the HIP library both consume what it returns.
Every generator is deterministic in its seed (NumPy PCG64, fixed draw order).

Layouts (all float32, structure-of-arrays):

* quadruples: ``src`` and ``dst`` of shape (8, n), planes
  ``xM yM xN yN xP yP xQ yQ`` (point order M, N, P, Q as in the ACA/SKS
  derivations: M, N, P are the anchors, Q the fourth point);
* correspondence sets: ``corr`` of shape (4, n), planes ``x1 y1 x2 y2``; a batch
  of sets is the concatenation with an int64 prefix array ``off`` (n_pairs + 1);
* patches: ``img`` and ``tgt`` of shape (B, 128, 128).

The workloads follow the shapes of the paper's experiments: 640x480 frames for
the correspondence problems (RANSAC experiment setup) and 128x128 grey patches
for the 4-point-offset pipeline (deep homography experiment setup).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FRAME_W = 640.0
FRAME_H = 480.0
CHUNK = 1 << 20            # quadruples per independently seeded chunk
W_MIN = 0.1                # reject perspective draws giving w < W_MIN on any point


def _random_similarity_persp(rng, m, centre=None):
    """Draw m random ground-truth homographies as (m, 3, 3) float64.

    Similarity: scale U[0.5, 2], rotation U[-pi, pi], translation U[-100, 100]^2;
    perspective row (h31, h32) U[-1e-3, 1e-3]^2 with h33 = 1. With ``centre`` the
    matrix is conjugated by the translation to that point (the map acts about the
    frame centre)."""
    s = rng.uniform(0.5, 2.0, m)
    th = rng.uniform(-math.pi, math.pi, m)
    t = rng.uniform(-100.0, 100.0, (m, 2))
    p = rng.uniform(-1e-3, 1e-3, (m, 2))
    H = np.zeros((m, 3, 3))
    H[:, 0, 0] = s * np.cos(th)
    H[:, 0, 1] = -s * np.sin(th)
    H[:, 1, 0] = s * np.sin(th)
    H[:, 1, 1] = s * np.cos(th)
    H[:, 0, 2] = t[:, 0]
    H[:, 1, 2] = t[:, 1]
    H[:, 2, 0] = p[:, 0]
    H[:, 2, 1] = p[:, 1]
    H[:, 2, 2] = 1.0
    if centre is not None:
        cx, cy = centre
        T = np.array([[1.0, 0.0, cx], [0.0, 1.0, cy], [0.0, 0.0, 1.0]])
        Ti = np.array([[1.0, 0.0, -cx], [0.0, 1.0, -cy], [0.0, 0.0, 1.0]])
        H = T @ H @ Ti
    return H


def _apply(H, x, y):
    """Project points (x, y) (shape (m, k)) under per-row H (m, 3, 3)."""
    u = H[:, 0, 0, None] * x + H[:, 0, 1, None] * y + H[:, 0, 2, None]
    v = H[:, 1, 0, None] * x + H[:, 1, 1, None] * y + H[:, 1, 2, None]
    w = H[:, 2, 0, None] * x + H[:, 2, 1, None] * y + H[:, 2, 2, None]
    return u, v, w


def _quad_chunk(seed, chunk, m, degenerate_every, base_index, with_h=False):
    rng = np.random.default_rng([seed, chunk])
    x = rng.uniform(0.0, FRAME_W, (m, 4))
    y = rng.uniform(0.0, FRAME_H, (m, 4))
    H = _random_similarity_persp(rng, m)
    # redraw the perspective row until every point has w >= W_MIN
    for _ in range(1000):
        _, _, w = _apply(H, x, y)
        bad = np.nonzero(w.min(axis=1) < W_MIN)[0]
        if bad.size == 0:
            break
        H[bad, 2, 0:2] = rng.uniform(-1e-3, 1e-3, (bad.size, 2))
    else:  # pragma: no cover - probability ~0
        raise RuntimeError("perspective rejection did not converge")
    labels = np.zeros(m, dtype=np.uint8)
    if degenerate_every:
        gidx = base_index + np.arange(m)
        sel = np.nonzero(gidx % degenerate_every == 0)[0]
        if sel.size:
            k = sel.size
            tri = rng.integers(0, 4, k)          # which point is moved onto the line
            lam = rng.uniform(-0.5, 1.5, k)      # position along the line of the other two
            off = rng.uniform(-1e-3, 1e-3, k)    # perpendicular offset in px
            others = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
            # the moved vertex is `tri`; the line runs through two of the other three
            pick = rng.integers(0, 3, (k, 2))
            pick[:, 1] = (pick[:, 0] + 1 + rng.integers(0, 2, k)) % 3
            a = others[tri, pick[:, 0]]
            b = others[tri, pick[:, 1]]
            ax, ay = x[sel, a], y[sel, a]
            bx, by = x[sel, b], y[sel, b]
            dx, dy = bx - ax, by - ay
            L = np.hypot(dx, dy)
            nx, ny = -dy / L, dx / L
            x[sel, tri] = ax + lam * dx + off * nx
            y[sel, tri] = ay + lam * dy + off * ny
            labels[sel] = 1
    u, v, w = _apply(H, x, y)
    noise = rng.normal(0.0, 0.5, (m, 4, 2))
    xd = u / w + noise[:, :, 0]
    yd = v / w + noise[:, :, 1]
    src = np.empty((8, m), np.float32)
    dst = np.empty((8, m), np.float32)
    src[0::2] = x.T
    src[1::2] = y.T
    dst[0::2] = xd.T
    dst[1::2] = yd.T
    if with_h:
        return src, dst, labels, H
    return src, dst, labels


def quadruples(n, seed, degenerate_every=0, chunks=None):
    """Quadruple workload (solver configs).

    Per quadruple, independently: four source points uniform in the 640x480
    frame; a random similarity with perspective row (see
    ``_random_similarity_persp``), perspective redrawn while any point has
    w < 0.1; targets = projection + N(0, 0.5^2) px noise; both rounded to fp32.
    With ``degenerate_every = k`` every quadruple whose global index is a
    multiple of k gets one source point moved onto the line through two others,
    within 1e-3 px (targets recomputed), and ``labels`` = 1 there.

    Chunks of ``CHUNK`` quadruples are seeded ``(seed, chunk)`` so any chunk can
    be regenerated alone. Returns (src, dst, labels)."""
    n = int(n)
    src = np.empty((8, n), np.float32)
    dst = np.empty((8, n), np.float32)
    lab = np.empty(n, np.uint8)
    nchunks = (n + CHUNK - 1) // CHUNK
    todo = range(nchunks) if chunks is None else chunks
    for c in todo:
        lo = c * CHUNK
        m = min(CHUNK, n - lo)
        s, d, l = _quad_chunk(seed, c, m, degenerate_every, lo)
        src[:, lo:lo + m] = s
        dst[:, lo:lo + m] = d
        lab[lo:lo + m] = l
    return src, dst, lab


def quadruple_chunk(seed, chunk, degenerate_every=0, m=CHUNK, with_h=False):
    """Chunk ``chunk`` (quadruples chunk*CHUNK ... + m) of ``quadruples(n, seed,
    degenerate_every)`` alone, without drawing the others; with ``with_h`` also
    the ground-truth homographies (m, 3, 3) drawn for it."""
    return _quad_chunk(seed, chunk, m, degenerate_every, chunk * CHUNK, with_h)


def _quad_worker(args):
    seed, c, m, k, lo = args
    return c, _quad_chunk(seed, c, m, k, lo)


def quadruples_parallel(n, seed, degenerate_every=0, workers=8, out=None):
    """Same result as ``quadruples`` (bit for bit), chunks drawn in a process pool."""
    import multiprocessing as mp
    n = int(n)
    if out is None:
        src = np.empty((8, n), np.float32)
        dst = np.empty((8, n), np.float32)
    else:
        src, dst = out
    lab = np.empty(n, np.uint8)
    nchunks = (n + CHUNK - 1) // CHUNK
    jobs = [(seed, c, min(CHUNK, n - c * CHUNK), degenerate_every, c * CHUNK) for c in range(nchunks)]
    if workers <= 1 or nchunks <= 1:
        for job in jobs:
            c, (s, d, l) = _quad_worker(job)
            lo = c * CHUNK
            src[:, lo:lo + s.shape[1]] = s
            dst[:, lo:lo + s.shape[1]] = d
            lab[lo:lo + s.shape[1]] = l
        return src, dst, lab
    ctx = mp.get_context("fork")
    pool = ctx.Pool(max(1, min(workers, nchunks)))
    try:
        for c, (s, d, l) in pool.imap_unordered(_quad_worker, jobs):
            lo = c * CHUNK
            m = s.shape[1]
            src[:, lo:lo + m] = s
            dst[:, lo:lo + m] = d
            lab[lo:lo + m] = l
        pool.close()      # let the workers exit on their own (no terminate signal)
    except BaseException:
        pool.terminate()
        raise
    finally:
        pool.join()
    return src, dst, lab


# A planar target in object units (say mm): points M, N, P, Q of a calibration
# board, as in the known-pattern setting of the simplified SK.
PATTERN = np.array([20.0, 30.0, 180.0, 25.0, 35.0, 140.0, 170.0, 150.0])


def _pattern_chunk(seed, chunk, m, obj):
    rng = np.random.default_rng([seed, chunk, 0x5C])
    ox, oy = obj[0::2], obj[1::2]
    cx, cy = ox.mean(), oy.mean()
    x = np.broadcast_to(ox - cx, (m, 4))
    y = np.broadcast_to(oy - cy, (m, 4))
    H = _random_similarity_persp(rng, m)
    for _ in range(1000):
        _, _, w = _apply(H, x, y)
        bad = np.nonzero(w.min(axis=1) < W_MIN)[0]
        if bad.size == 0:
            break
        H[bad, 2, 0:2] = rng.uniform(-1e-3, 1e-3, (bad.size, 2))
    else:  # pragma: no cover - probability ~0
        raise RuntimeError("perspective rejection did not converge")
    u, v, w = _apply(H, x, y)
    noise = rng.normal(0.0, 0.5, (m, 4, 2))
    dst = np.empty((8, m), np.float32)
    dst[0::2] = (u / w + FRAME_W / 2 + noise[:, :, 0]).T
    dst[1::2] = (v / w + FRAME_H / 2 + noise[:, :, 1]).T
    return dst


def _pattern_worker(args):
    seed, c, m, obj = args
    return c, _pattern_chunk(seed, c, m, obj)


def pattern_images(n, seed, obj=PATTERN, workers=1):
    """Images of one planar pattern ``obj`` (8 numbers M N P Q, object units):
    per image a random similarity with perspective row (as for quadruples),
    acting about the pattern's centroid and placed at the frame centre, the
    perspective redrawn while a point has w < 0.1, plus N(0, 0.5^2) px noise;
    float32 planes (8, n). Chunks of ``CHUNK`` images are seeded
    ``(seed, chunk)``; ``workers`` > 1 draws them in a process pool (same
    result)."""
    n = int(n)
    obj = np.asarray(obj, np.float64)
    dst = np.empty((8, n), np.float32)
    jobs = [(seed, c, min(CHUNK, n - c * CHUNK), obj) for c in range((n + CHUNK - 1) // CHUNK)]
    if workers <= 1 or len(jobs) <= 1:
        results = map(_pattern_worker, jobs)
        pool = None
    else:
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(max(1, min(workers, len(jobs))))
        results = pool.imap_unordered(_pattern_worker, jobs)
    try:
        for c, d in results:
            dst[:, c * CHUNK:c * CHUNK + d.shape[1]] = d
        if pool is not None:
            pool.close()
    except BaseException:
        if pool is not None:
            pool.terminate()
        raise
    finally:
        if pool is not None:
            pool.join()
    return dst


@dataclasses.dataclass
class CorrSet:
    corr: np.ndarray      # (4, n) float32: x1 y1 x2 y2
    inlier: np.ndarray    # (n,) bool ground-truth labels
    H_true: np.ndarray    # (3, 3) float64


def _corr_set(rng, n, n_in):
    H = _random_similarity_persp(rng, 1, centre=(FRAME_W / 2, FRAME_H / 2))
    x1 = rng.uniform(0.0, FRAME_W, n)
    y1 = rng.uniform(0.0, FRAME_H, n)
    x2 = rng.uniform(0.0, FRAME_W, n)
    y2 = rng.uniform(0.0, FRAME_H, n)
    u, v, w = _apply(H, x1[None, :n_in], y1[None, :n_in])
    noise = rng.normal(0.0, 1.0, (2, n_in))
    x2[:n_in] = (u / w)[0] + noise[0]
    y2[:n_in] = (v / w)[0] + noise[1]
    perm = rng.permutation(n)
    corr = np.stack([x1, y1, x2, y2])[:, perm].astype(np.float32)
    inl = np.zeros(n, bool)
    inl[:n_in] = True
    return CorrSet(np.ascontiguousarray(corr), inl[perm], H[0])


def correspondences(n, inlier_ratio, seed):
    """One correspondence set in the 640x480 frame: round(ratio*n) inliers mapped
    by one random homography about the frame centre plus N(0, 1) px noise, the
    rest uniform outliers on both sides; order shuffled."""
    rng = np.random.default_rng([seed, 0])
    return _corr_set(rng, int(n), int(round(inlier_ratio * n)))


@dataclasses.dataclass
class CorrBatch:
    corr: np.ndarray      # (4, total) float32
    off: np.ndarray       # (n_pairs + 1,) int64
    inlier: np.ndarray    # (total,) bool
    ratio: np.ndarray     # (n_pairs,) float64
    H_true: np.ndarray    # (n_pairs, 3, 3)


def correspondence_batch(n_pairs, seed, n_min=100, n_max=8000, r_min=0.1, r_max=0.9):
    """Uneven batch of correspondence sets: N_p ~ U{n_min..n_max}, inlier ratio
    U[r_min, r_max]; pair p drawn from its own stream (seed, p + 1)."""
    top = np.random.default_rng([seed, 0])
    ns = top.integers(n_min, n_max + 1, n_pairs)
    rs = top.uniform(r_min, r_max, n_pairs)
    off = np.zeros(n_pairs + 1, np.int64)
    off[1:] = np.cumsum(ns)
    corr = np.empty((4, int(off[-1])), np.float32)
    inl = np.empty(int(off[-1]), bool)
    Hs = np.empty((n_pairs, 3, 3))
    for p in range(n_pairs):
        rng = np.random.default_rng([seed, p + 1])
        cs = _corr_set(rng, int(ns[p]), int(round(rs[p] * ns[p])))
        corr[:, off[p]:off[p + 1]] = cs.corr
        inl[off[p]:off[p + 1]] = cs.inlier
        Hs[p] = cs.H_true
    return CorrBatch(corr, off, inl, rs, Hs)


def integer_identity_batch(sizes, seed, inlier_ratio=0.4, side=16):
    """Pairs whose inliers are exact: integer points in [0, side)^2 with
    x2 = x1 for a fraction inlier_ratio of each pair, and x2 another integer
    point (x2 != x1) for the rest. Every quantity a sample of four inliers
    produces is then an integer small enough for exact float arithmetic, so an
    inlier's transfer error under such a sample's homography is exactly 0.
    Pair p is drawn from the stream (seed, p + 1); returns a CorrBatch."""
    ns = np.asarray(sizes, np.int64)
    off = np.zeros(len(ns) + 1, np.int64)
    off[1:] = np.cumsum(ns)
    corr = np.empty((4, int(off[-1])), np.float32)
    inl = np.empty(int(off[-1]), bool)
    for p, n in enumerate(ns):
        rng = np.random.default_rng([seed, p + 1])
        x1 = rng.integers(0, side, (2, int(n)))
        is_in = rng.random(int(n)) < inlier_ratio
        x2 = rng.integers(0, side, (2, int(n)))
        same = (x2 == x1).all(axis=0) & ~is_in
        x2[0, same] = (x1[0, same] + 1) % side          # outliers never coincide
        x2[:, is_in] = x1[:, is_in]
        corr[:, off[p]:off[p + 1]] = np.concatenate([x1, x2]).astype(np.float32)
        inl[off[p]:off[p + 1]] = is_in
    return CorrBatch(corr, off, inl, np.full(len(ns), inlier_ratio), np.tile(np.eye(3), (len(ns), 1, 1)))


def _blur_1d(a, axis, sigma, radius):
    k = np.exp(-0.5 * (np.arange(-radius, radius + 1) / sigma) ** 2)
    k /= k.sum()
    n = a.shape[axis] - 2 * radius
    out = np.zeros(a.shape[:axis] + (n,) + a.shape[axis + 1:], np.float64)
    for i, kv in enumerate(k):
        sl = [slice(None)] * a.ndim
        sl[axis] = slice(i, i + n)
        out += kv * a[tuple(sl)]
    return out


@dataclasses.dataclass
class PatchBatch:
    img: np.ndarray       # (B, S, S) float32
    tgt: np.ndarray       # (B, S, S) float32
    offsets: np.ndarray   # (B, 4, 2) float32, corner order TL, TR, BR, BL
    shift: np.ndarray     # (B, 2) int64, integer displacement of the target crop


def patches(B, seed, size=128, sigma=4.0, max_shift=16, max_offset=32.0):
    """Smooth random patches for the 4-point-offset pipeline.

    A field of N(0, 1) noise is blurred by a separable Gaussian (sigma = 4 px,
    truncated at 3 sigma); the source patch is its centre crop and the target
    patch a crop displaced by an integer shift in U{-16..16}^2 (a second view of
    the same scene). Each patch is standardised. Corner offsets are
    U[-32, 32] px per coordinate."""
    rng = np.random.default_rng([seed, 0])
    radius = int(math.ceil(3 * sigma))
    big = size + 2 * max_shift
    canvas = big + 2 * radius
    img = np.empty((B, size, size), np.float32)
    tgt = np.empty((B, size, size), np.float32)
    shift = rng.integers(-max_shift, max_shift + 1, (B, 2))
    offsets = rng.uniform(-max_offset, max_offset, (B, 4, 2)).astype(np.float32)
    step = 64
    for b0 in range(0, B, step):
        b1 = min(B, b0 + step)
        noise = rng.normal(0.0, 1.0, (b1 - b0, canvas, canvas))
        field = _blur_1d(_blur_1d(noise, 1, sigma, radius), 2, sigma, radius)
        for i in range(b1 - b0):
            b = b0 + i
            a = field[i, max_shift:max_shift + size, max_shift:max_shift + size]
            sy, sx = max_shift + shift[b, 1], max_shift + shift[b, 0]
            t = field[i, sy:sy + size, sx:sx + size]
            img[b] = ((a - a.mean()) / a.std()).astype(np.float32)
            tgt[b] = ((t - t.mean()) / t.std()).astype(np.float32)
    return PatchBatch(img, tgt, offsets, shift)


# The five workloads as named configurations -------------------------------

def config0():
    """4096 quadruples, seed 0, no planted degeneracies."""
    return quadruples(4096, 0)


def config1(n=1 << 26, parallel=True, workers=8):
    """2^26 quadruples, seed 1, 1 % near-degenerate (index % 100 == 0)."""
    if parallel:
        return quadruples_parallel(n, 1, degenerate_every=100, workers=workers)
    return quadruples(n, 1, degenerate_every=100)


def config2():
    """N = 2000 correspondences, 30 % inliers, seed 2."""
    return correspondences(2000, 0.3, 2)


def config3(n_pairs=512):
    """512 uneven pairs, N ~ U{100..8000}, ratio U[0.1, 0.9], seed 3."""
    return correspondence_batch(n_pairs, 3)


def config4(B=1024):
    """1024 smooth 128x128 patches with corner offsets, seed 4."""
    return patches(B, 4)
