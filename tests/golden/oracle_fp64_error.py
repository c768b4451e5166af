"""Float64 error of the oracle's solvers against exact rational arithmetic,
per workload.

For each workload, 512 problems are drawn at fixed positions (seeded), the
oracle's float64 solver (ACA in its structured order, SKS, Algorithm 1 on the
config-4 square) is evaluated, and its error against the exact rational DLT
solution (``homography.exact_h``) is measured as the Frobenius distance of the
normalised, sign-fixed matrices. Reported: max, p99 and median. The float32
emulation of ACA (every operation rounded to float) is listed as context.

Run as a script to (re)write ``oracle_fp64_error.json`` next to this file; the
table is stored so that a reader (and the benchmark's report) can quote it
without recomputing exact arithmetic. Calls only the oracle and the input
generators.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth                                     # noqa: E402
from oracle import homography as hg              # noqa: E402
from oracle import ransac as oref                # noqa: E402

N_SETS = 512
JSON = os.path.join(HERE, "oracle_fp64_error.json")


def _pick(n, k, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(k, n), replace=False))


def _stats(e):
    e = np.asarray(e, np.float64)
    return dict(n=int(e.size), max=float(e.max()), p99=float(np.quantile(e, 0.99)),
                median=float(np.median(e)))


def _errors(src, dst, sel, solvers):
    """Errors of each solver (name -> H (n, 3, 3)) against exact_h on columns sel."""
    out = {k: [] for k in solvers}
    for i in sel:
        Hx = hg.exact_h(src[:, i], dst[:, i])
        for k, H in solvers.items():
            out[k].append(float(hg.herr(H[i], Hx)))
    return out


def _hyp_quads(corr, n_hyp, seed, pair):
    """The sampled quadruples of a RANSAC pair's hypotheses and their validity."""
    idx, _, _, valid = oref.hypotheses(corr, n_hyp, seed, pair)
    src = np.stack([corr[c, idx[k]] for k in range(4) for c in (0, 1)])
    dst = np.stack([corr[c, idx[k]] for k in range(4) for c in (2, 3)])
    return src, dst, valid


def table(n_sets=N_SETS):
    rows = {}
    # config 0: 4096 quadruples, seed 0
    s, d, _ = synth.config0()
    sel = _pick(s.shape[1], n_sets, 100)
    s64, d64 = s.astype(np.float64), d.astype(np.float64)
    e = _errors(s, d, sel, {"aca64": hg.aca64(s64, d64), "sks64": hg.sks64(s64, d64),
                            "aca32": hg.aca64(s, d)})
    rows["config0_aca64"] = _stats(e["aca64"])
    rows["config0_sks64"] = _stats(e["sks64"])
    rows["config0_aca_float32_emulation"] = _stats(e["aca32"])
    # config 1: chunks 0 and 63 of the 2^26 batch (seed 1, 1 % planted
    # near-degenerate sets); non-flagged and flagged sets separately
    src, dst = [], []
    for c in (0, 63):
        a, b, _ = synth.quadruple_chunk(1, c, 100, m=1 << 16)
        src.append(a)
        dst.append(b)
    s, d = np.concatenate(src, 1), np.concatenate(dst, 1)
    flags = hg.degeneracy_flags(s, d)
    s64, d64 = s.astype(np.float64), d.astype(np.float64)
    H = {"aca64": hg.aca64(s64, d64), "sks64": hg.sks64(s64, d64)}
    for name, mask in (("unflagged", flags == 0), ("flagged", flags != 0)):
        cols = np.nonzero(mask)[0]
        sel = cols[_pick(cols.size, n_sets, 101)]
        e = _errors(s, d, sel, H)
        rows[f"config1_{name}_aca64"] = _stats(e["aca64"])
        rows[f"config1_{name}_sks64"] = _stats(e["sks64"])
    # config 2: the 4096 hypotheses of the single pair (valid samples)
    cs = synth.config2()
    s, d, valid = _hyp_quads(cs.corr, 4096, 2, 0)
    cols = np.nonzero(valid)[0]
    sel = cols[_pick(cols.size, n_sets, 102)]
    e = _errors(s, d, sel, {"aca64": hg.aca64(s.astype(np.float64), d.astype(np.float64))})
    rows["config2_hypotheses_aca64"] = _stats(e["aca64"])
    # config 3: hypotheses of 16 pairs spread over the batch, 32 valid each
    cb = synth.config3()
    errs = []
    for k, p in enumerate(range(0, 512, 32)):
        a, b = cb.off[p], cb.off[p + 1]
        s, d, valid = _hyp_quads(cb.corr[:, a:b], 1024, 3, p)
        cols = np.nonzero(valid)[0]
        sel = cols[_pick(cols.size, n_sets // 16, 200 + k)]
        errs += _errors(s, d, sel, {"aca64": hg.aca64(s.astype(np.float64),
                                                      d.astype(np.float64))})["aca64"]
    rows["config3_hypotheses_aca64"] = _stats(errs)
    # config 4: Algorithm 1 on the 127 x 127 square with the 1024 patches' offsets
    pb = synth.patches(1024, 4, size=8)   # config-4 offsets (drawn before the image field)
    off = pb.offsets.astype(np.float64)                           # (B, 4, 2): TL TR BR BL
    src = np.array(hg.rect_corners(0.0, 0.0, 127.0, 1.0))          # M N P Q = TL TR BL BR
    tl, tr, br, bl = (off[:, k] for k in range(4))
    q = np.stack([tl[:, 0], tl[:, 1], 127 + tr[:, 0], tr[:, 1], bl[:, 0], 127 + bl[:, 1],
                  127 + br[:, 0], 127 + br[:, 1]])
    H = hg.aca_rect64(0.0, 0.0, 127.0, 1.0, q, square=True)
    S = np.repeat(src[:, None], q.shape[1], axis=1)
    sel = _pick(q.shape[1], n_sets, 104)
    rows["config4_rect_aca64"] = _stats(_errors(S, q, sel, {"r": H})["r"])
    return rows


if __name__ == "__main__":
    t = table()
    with open(JSON, "w") as f:
        json.dump(t, f, indent=1, sort_keys=True)
        f.write("\n")
    for k, v in t.items():
        print(f"{k:40s} n={v['n']:4d} max={v['max']:.2e} p99={v['p99']:.2e} median={v['median']:.2e}")
