"""Hypothesis sampling for RANSAC (oracle; test infrastructure only).

The paper's RANSAC draws random 4-point subsets (RANSAC pipeline description in
the experiments) but does not name a generator. This implementation uses a
counter-based generator so that every hypothesis can be drawn independently and
identically on CPU and GPU:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC 2011): 10 rounds of two 32x32->64 multiplies on a 4-word
  counter with a 2-word key bumped by the Weyl constants between rounds.
  Key = the 64-bit seed (low word first); counter = (hypothesis, pair, 0, 0).
* Floyd's subset algorithm (Bentley and Floyd, "A sample of brilliance",
  CACM 1987) for 4 distinct indices of N: for j = N-4 .. N-1 draw t uniform in
  [0, j] and take t unless already taken, else j. The uniform draw is the
  multiply-high t = (r * (j + 1)) >> 32 of one 32-bit Philox output word.
  The order of choice gives the roles M, N, P, Q.

Pins: the published Philox4x32-10 known-answer vectors (tests/golden), brute
force over every Floyd outcome for small N, distinctness and uniformity. The
mapping from words to indices is this implementation's own choice and has no
external reference beyond those properties.
"""
from __future__ import annotations

import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32-10 on uint32 arrays: ``ctr`` (4, ...) and ``key`` (2, ...),
    broadcast together. Returns (4, ...) uint32."""
    arrs = np.broadcast_arrays(*[np.asarray(x, np.uint64) for x in (*ctr, *key)])
    c = [a & np.uint64(MASK32) for a in arrs[:4]]
    k0 = arrs[4] & np.uint64(MASK32)
    k1 = arrs[5] & np.uint64(MASK32)
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + np.uint64(PHILOX_W0)) & np.uint64(MASK32)
            k1 = (k1 + np.uint64(PHILOX_W1)) & np.uint64(MASK32)
        p0 = m0 * c[0]                      # exact: < 2^64
        p1 = m1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK32)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack([x.astype(np.uint32) for x in c])


def seed_key(seed):
    """Split a 64-bit seed into the two Philox key words (low, high)."""
    seed = int(seed) & ((1 << 64) - 1)
    return seed & MASK32, seed >> 32


def floyd4(r, n):
    """Floyd's algorithm for 4 distinct indices of ``n`` from four uint32 words
    ``r`` (4, ...) ; ``n`` broadcastable (>= 4). Returns (4, ...) int64 in
    order of choice."""
    r = np.asarray(r, np.uint64)
    n = np.asarray(n, np.int64)
    out = []
    for i in range(4):
        j = n - 4 + i
        t = ((r[i] * (j + 1).astype(np.uint64)) >> np.uint64(32)).astype(np.int64)
        taken = np.zeros(np.broadcast(t, n).shape, bool)
        for prev in out:
            taken |= prev == t
        out.append(np.where(taken, j, t))
    return np.stack(out)


def sample_indices(n_pts, n_hyp, seed, pair=0):
    """The 4 indices (4, n_hyp) drawn for hypotheses 0..n_hyp-1 of one pair."""
    h = np.arange(n_hyp, dtype=np.uint64)
    k0, k1 = seed_key(seed)
    r = philox4x32_10((h, np.uint64(pair), np.uint64(0), np.uint64(0)), (k0, k1))
    return floyd4(r, n_pts)
