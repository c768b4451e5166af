"""Pins for the oracle's hypothesis sampler (CPU only)."""
import itertools
import os
from collections import Counter

import numpy as np

from oracle import sampling

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def load_kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        rows.append([int(t, 16) for t in line.split()])
    return rows


def test_philox_known_answers():
    rows = load_kat()
    assert len(rows) == 3
    for r in rows:
        out = sampling.philox4x32_10(r[0:4], r[4:6])
        assert [int(x) for x in out] == r[6:10]


def test_philox_vectorised_matches_elementwise():
    ctr = (np.arange(50, dtype=np.uint64), np.uint64(7), np.uint64(0), np.uint64(0))
    out = sampling.philox4x32_10(ctr, sampling.seed_key(0x123456789ABCDEF))
    for i in range(0, 50, 7):
        o = sampling.philox4x32_10((i, 7, 0, 0), sampling.seed_key(0x123456789ABCDEF))
        assert np.array_equal(out[:, i], o)


def _word_for(t, j):
    # smallest 32-bit word whose multiply-high maps to t in [0, j]
    return -((-t << 32) // (j + 1))


def test_floyd_exhaustive_uniform():
    # every combination of the four uniform draws, each equally likely, must give
    # every 4-subset the same number of times (24 = 4! orders of the draws)
    for n in (4, 5, 6, 7, 9):
        counts = Counter()
        ranges = [range(j + 1) for j in range(n - 4, n)]
        for ts in itertools.product(*ranges):
            r = np.array([_word_for(t, j) for t, j in zip(ts, range(n - 4, n))], np.uint64)
            idx = sampling.floyd4(r[:, None], n)[:, 0]
            assert len(set(idx.tolist())) == 4 and idx.min() >= 0 and idx.max() < n
            counts[frozenset(idx.tolist())] += 1
        from math import comb
        assert len(counts) == comb(n, 4)
        assert set(counts.values()) == {n * (n - 1) * (n - 2) * (n - 3) // comb(n, 4)}


def test_floyd_word_mapping_boundaries():
    # word 0 -> 0 and word 2^32-1 -> j for every j
    for n in (4, 10, 2000, 8000, 1 << 30):
        j = np.array([n - 4, n - 3, n - 2, n - 1], np.int64)
        lo = sampling.floyd4(np.zeros((4, 1), np.uint64), n)[:, 0]
        hi = ((np.uint64(0xFFFFFFFF) * (j + 1).astype(np.uint64)) >> np.uint64(32)).astype(np.int64)
        assert np.array_equal(hi, j)
        assert lo[0] == 0 and len(set(lo.tolist())) == 4


def test_sample_indices_distinct_and_uniform():
    n, h = 2000, 200000
    idx = sampling.sample_indices(n, h, seed=2)
    assert idx.shape == (4, h)
    s = np.sort(idx, axis=0)
    assert np.all(np.diff(s, axis=0) > 0)
    assert idx.min() >= 0 and idx.max() < n
    # each index is in a sample with probability 4/n: chi-square over 2000 cells
    cnt = np.bincount(idx.ravel(), minlength=n)
    e = 4 * h / n
    chi2 = ((cnt - e) ** 2 / e).sum()
    assert 1700 < chi2 < 2300          # dof 1999, sd ~63
    # different pairs and seeds give different streams
    assert not np.array_equal(idx[:, :100], sampling.sample_indices(n, 100, seed=2, pair=1))
    assert not np.array_equal(idx[:, :100], sampling.sample_indices(n, 100, seed=3))
