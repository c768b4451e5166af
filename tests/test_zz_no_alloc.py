"""hg_ransac_noalloc (the library's own static workspace) against hg_ransac
(caller workspace): identical outputs, bit for bit, on two calls in a row, the
second with fewer points and hypotheses; hypothesis counts above the
workspace's maximum are refused before any launch."""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu
TAU = 3.0


def _outputs(n, n_hyp):
    return [torch.full((9,), -1.0, device="cuda"),
            torch.full((1,), -1, dtype=torch.int32, device="cuda"),
            torch.full((1,), -1, dtype=torch.int32, device="cuda"),
            torch.full((n,), 7, dtype=torch.uint8, device="cuda"),
            torch.full((n_hyp,), -1, dtype=torch.int32, device="cuda")]


def _call(name, corr, n_hyp, seed):
    from paper_2402_18008_amd import _abi
    L = _abi.lib()
    n, ld = corr.shape[1], corr.stride(0)
    o = _outputs(n, n_hyp)
    args = [corr.data_ptr(), n, ld, n_hyp, TAU, seed] + [t.data_ptr() for t in o]
    s = torch.cuda.current_stream().cuda_stream
    if name == "hg_ransac":
        ws = torch.empty(L.hg_ransac_ws_bytes(n, n_hyp), dtype=torch.uint8, device="cuda")
        st = L.hg_ransac(*args, ws.data_ptr(), ws.numel(), s)
    else:
        st = L.hg_ransac_noalloc(*args, s)
    assert st == 0, L.hg_last_error()
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in o]


def test_noalloc_matches_caller_workspace():
    require_gpu()
    # first call: the 2000-point, 4096-hypothesis pair; second: smaller
    cases = [(synth.config2().corr, 4096, 2), (synth.correspondences(700, 0.4, 5).corr, 1000, 9)]
    for corr_np, n_hyp, seed in cases:
        corr = torch.from_numpy(corr_np).cuda()
        announce(f"hg_ransac_noalloc n={corr.shape[1]} hyps={n_hyp}")
        got = _call("hg_ransac_noalloc", corr, n_hyp, seed)
        ref = _call("hg_ransac", corr, n_hyp, seed)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
        assert int(got[1][0]) == int(got[4].max()) and int(got[3].sum()) == int(got[1][0])


def test_noalloc_rejects_too_many_hypotheses():
    require_gpu()
    from paper_2402_18008_amd import _abi
    L = _abi.lib()
    corr = torch.from_numpy(synth.correspondences(100, 0.5, 3).corr).cuda()
    o = _outputs(100, 16385)
    st = L.hg_ransac_noalloc(corr.data_ptr(), 100, 100, 16385, TAU, 1,
                             *[t.data_ptr() for t in o], torch.cuda.current_stream().cuda_stream)
    assert st == _abi.HG_EINVAL and b"16384" in L.hg_last_error()
