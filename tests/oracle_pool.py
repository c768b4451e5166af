"""Oracle RANSAC references of many pairs, computed in a pool of CPU
processes (spawned: the workers import numpy and the oracle only, never the
GPU library)."""
import multiprocessing as mp
import os

import numpy as np

from oracle import ransac as oref


def _ref(job):
    corr, n_hyp, tau, seed, pair = job
    return pair, oref.ransac_ref(corr, n_hyp, tau, seed, pair=pair)


def ransac_refs(corr, off, n_hyp, tau, seed, workers=None):
    """ransac_ref of every pair p (points off[p]:off[p+1] of corr), as a list."""
    n_pairs = len(off) - 1
    jobs = [(np.ascontiguousarray(corr[:, off[p]:off[p + 1]]), n_hyp, tau, seed, p)
            for p in range(n_pairs)]
    jobs.sort(key=lambda j: -j[0].shape[1])        # largest first, for balance
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    out = [None] * n_pairs
    with mp.get_context("spawn").Pool(workers) as pool:
        for p, ref in pool.imap_unordered(_ref, jobs, chunksize=1):
            out[p] = ref
    return out
