"""HO-SVD refit on inliers on the GPU against the oracle (parity tests).

Bar: per pair, the number of points used is exact; H agrees with the oracle's
float64 HO-SVD (QR + SVD of the 2n x 3 reduced matrix) within 1e-6 after
Frobenius normalisation and sign fixing (the GPU forms the 3 x 3 Gram matrix
in double and rounds H to float; the float rounding alone is ~6e-8); pairs
with fewer than 4 selected points give H = 0 with bit2 set."""
import numpy as np
import pytest
import torch

import synth
from oracle import homography as hg
from oracle import refit
from tests.gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-6


def gpu_refit(corr, off, mask):
    import paper_2402_18008_amd as hgpu
    C = torch.from_numpy(np.ascontiguousarray(corr)).cuda()
    O = torch.from_numpy(np.asarray(off, np.int64)).cuda()
    M = None if mask is None else torch.from_numpy(np.asarray(mask, np.uint8)).cuda()
    H, used, flags = hgpu.hg_refit_ho(C, O, M)
    torch.cuda.synchronize()
    return H.cpu().numpy().reshape(-1, 3, 3), used.cpu().numpy(), flags.cpu().numpy()


def check(corr, off, mask, Hg, ug, fg, pairs=None, label=""):
    P = len(off) - 1
    pairs = range(P) if pairs is None else pairs
    full = np.ones(corr.shape[1], np.uint8) if mask is None else mask
    worst = 0.0
    for p in pairs:
        a, b = int(off[p]), int(off[p + 1])
        sel = np.nonzero(full[a:b])[0] + a
        assert ug[p] == sel.size, (label, p)
        if sel.size < 4:
            assert fg[p] == 4 and not Hg[p].any(), (label, p)
            continue
        Ho = refit.ho_svd(*(corr[k, sel].astype(np.float64) for k in range(4)))
        assert fg[p] == 0, (label, p)
        e = hg.herr(Hg[p].astype(np.float64), Ho)
        worst = max(worst, e)
        assert e <= TOL, (label, p, e)
    return worst


def test_refit_ground_truth_masks():
    require_gpu()
    b = synth.correspondence_batch(64, 41, n_min=100, n_max=2000)
    mask = b.inlier.astype(np.uint8)
    announce("refit_ho 64 pairs, ground-truth inlier masks")
    Hg, ug, fg = gpu_refit(b.corr, b.off, mask)
    w = check(b.corr, b.off, mask, Hg, ug, fg, label="gt")
    print("refit worst herr", w)
    # the same call checked against a host copy of the offsets
    import paper_2402_18008_amd as hgpu
    C = torch.from_numpy(np.ascontiguousarray(b.corr)).cuda()
    O = torch.from_numpy(b.off).cuda()
    M = torch.from_numpy(mask).cuda()
    H2, u2, f2 = hgpu.hg_refit_ho(C, O, M, off_host=b.off)
    torch.cuda.synchronize()
    assert np.array_equal(H2.cpu().numpy().reshape(-1, 3, 3), Hg)
    assert np.array_equal(u2.cpu().numpy(), ug) and np.array_equal(f2.cpu().numpy(), fg)
    bad = b.off.copy()
    bad[3], bad[4] = bad[4], bad[3]
    with pytest.raises(ValueError):
        hgpu.hg_refit_ho(C, O, M, off_host=bad)
    with pytest.raises(ValueError):
        hgpu.hg_refit_ho(C, O, M, off_host=b.off[:-1])


def test_refit_masks_small_sets_and_no_mask():
    require_gpu()
    b = synth.correspondence_batch(10, 42, n_min=4, n_max=300)
    rng = np.random.default_rng(5)
    mask = (rng.random(b.corr.shape[1]) < 0.5).astype(np.uint8)
    mask[b.off[1]:b.off[2]] = 0                       # nothing selected
    mask[b.off[2]:b.off[3]] = 0
    mask[b.off[2]:b.off[2] + 3] = 1                   # three points
    mask[b.off[3]:b.off[4]] = 0
    mask[b.off[3]:b.off[3] + 4] = 1                   # exactly four
    announce("refit_ho random masks, 0 / 3 / 4 points")
    Hg, ug, fg = gpu_refit(b.corr, b.off, mask)
    check(b.corr, b.off, mask, Hg, ug, fg, label="random")
    announce("refit_ho without a mask")
    Hg, ug, fg = gpu_refit(b.corr, b.off, None)
    check(b.corr, b.off, None, Hg, ug, fg, label="all")


def test_refit_reference_point_far_or_not_finite():
    """The kernel sums moments about each pair's first point, selected or not.
    An unselected first point far from the others (1e5 px away), or with
    non-finite coordinates, changes nothing: the result matches the oracle on
    the selected points."""
    require_gpu()
    b = synth.correspondence_batch(8, 43, n_min=200, n_max=600)
    corr = b.corr.copy()
    mask = b.inlier.astype(np.uint8)
    for p in range(8):
        a = int(b.off[p])
        mask[a] = 0
        if p % 2 == 0:
            corr[:, a] = np.float32(1e5)                   # far away
        else:
            corr[:, a] = [np.nan, np.inf, -np.inf, np.nan]  # not finite
    announce("refit_ho unselected first points far away / not finite")
    Hg, ug, fg = gpu_refit(corr, b.off, mask)
    check(corr, b.off, mask, Hg, ug, fg, label="reference point")


def test_refit_exact_points():
    """Noise-free correspondences (rounded to float) give back the generating
    homography."""
    require_gpu()
    rng = np.random.default_rng(6)
    n = 500
    cs = synth.correspondences(10, 0.5, 77)
    H = cs.H_true
    x = rng.uniform(0, 640, n)
    y = rng.uniform(0, 480, n)
    w = H[2, 0] * x + H[2, 1] * y + H[2, 2]
    u = (H[0, 0] * x + H[0, 1] * y + H[0, 2]) / w
    v = (H[1, 0] * x + H[1, 1] * y + H[1, 2]) / w
    corr = np.stack([x, y, u, v]).astype(np.float32)
    announce("refit_ho exact points n=500")
    Hg, ug, fg = gpu_refit(corr, [0, n], None)
    assert ug[0] == n and fg[0] == 0
    assert hg.herr(Hg[0].astype(np.float64), H) < 1e-5


def test_refit_config3_size_sampled():
    """512 uneven pairs (N ~ U{100..8000}, about 2.07M points) in one launch
    with the ground-truth inlier masks; 48 sampled pairs against the oracle."""
    require_gpu()
    announce("refit_ho config3 generating")
    b = synth.config3()
    mask = b.inlier.astype(np.uint8)
    announce("refit_ho config3 launch")
    Hg, ug, fg = gpu_refit(b.corr, b.off, mask)
    assert np.array_equal(ug, np.add.reduceat(mask.astype(np.int64), b.off[:-1]))
    pairs = np.random.default_rng(7).choice(len(b.off) - 1, 48, replace=False)
    w = check(b.corr, b.off, mask, Hg, ug, fg, pairs=pairs, label="config3")
    print("config3 refit worst herr", w)
