"""The oracle's own float64 error against exact rational arithmetic, per
workload (512 problems each; config 1 split into unflagged and flagged sets).

The table is recomputed here and must equal the stored one
(``tests/golden/oracle_fp64_error.json``, written by the script next to it),
and every float64 figure must be far below the 1e-5 tolerance that the GPU is
held to against this oracle."""
import json
import os

import numpy as np

from tests.golden import oracle_fp64_error as ofe


def test_oracle_fp64_error_per_config():
    t = ofe.table()
    with open(ofe.JSON) as f:
        stored = json.load(f)
    assert sorted(t) == sorted(stored)
    for k, v in t.items():
        s = stored[k]
        assert v["n"] == s["n"] >= 512, k
        for q in ("max", "p99", "median"):
            assert np.isclose(v[q], s[q], rtol=1e-6, atol=0.0), (k, q, v[q], s[q])
        print(f"{k:40s} max={v['max']:.2e} p99={v['p99']:.2e}")
        if "float32" in k:
            assert v["max"] > 1e-6          # single precision is visibly worse (context)
        elif "flagged" in k and "unflagged" not in k:
            assert v["max"] < 1e-10         # near-degenerate, still ~1e-12
        else:
            assert v["max"] < 1e-11
