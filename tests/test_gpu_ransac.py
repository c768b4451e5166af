"""RANSAC on the GPU against the oracle (parity tests).

Bar (integer results): the sampled hypotheses' validity is exact (up to
samples whose minimum triangle height lies within a relative 1e-3 of the
degeneracy threshold); every per-hypothesis count equals the oracle's float64
count except for points whose transfer error lies within 1e-4 px of the
threshold (it lies in the oracle's [count_lo, count_hi] at that band); the
best hypothesis is the lowest-index maximum of the GPU counts and equals the
oracle's wherever no exempt point can change the order; the winning H matches
the oracle's within 1e-5 (it is the same float64 ACA, scaled and rounded);
the mask equals the oracle's inlier set of that H outside the 1e-4 px band;
fused, plain and persistent forms agree bit for bit."""
import numpy as np
import pytest
import torch

import synth
from oracle import homography as hg
from oracle import ransac as oref
from tests.gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu
TAU = 3.0
BAND_PX = 1e-4      # counts are exact except points this close to the threshold


def to_np(d):
    return {k: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for k, v in d.items()}


def check_pair(corr, n_hyp, seed, got, pair=0, label="", ref=None):
    """Compare one pair's GPU results (numpy dict) with the oracle (ref: the
    pair's ransac_ref, if already computed)."""
    if ref is None:
        ref = oref.ransac_ref(corr, n_hyp, TAU, seed, pair=pair)
    idx = ref["idx"]
    src = np.stack([corr[c, idx[k]] for k in range(4) for c in (0, 1)])
    dst = np.stack([corr[c, idx[k]] for k in range(4) for c in (2, 3)])
    mh = hg.min_height(src, dst)
    borderline = np.abs(mh - hg.DELTA_PX) <= 1e-3 * hg.DELTA_PX
    counts = got["hyp_counts"].astype(np.int64)
    valid_o = ref["valid"]
    # validity: an invalid hypothesis reports 0; compare where not borderline
    nb = ~borderline
    gv = counts > 0
    assert not (gv & ~valid_o & nb).any(), f"{label}: GPU counted an invalid sample"
    ok = valid_o & nb
    lo, hi = ref["count_lo"], ref["count_hi"]
    bad = ok & ((counts < lo) | (counts > hi))
    if bad.any():
        j = np.nonzero(bad)[0][:8]
        # diagnostic: how far the mis-counted points lie from the threshold,
        # next to the float32 decision band of those hypotheses
        d = oref.transfer_error(ref["H32"][j], corr)
        band = oref.decision_band(ref["H32"][j], corr, TAU)
        near = np.abs(d - TAU)
        k = np.argsort(near, axis=1)[:, :3]
        raise AssertionError((label, j, counts[j], ref["counts"][j], lo[j], hi[j],
                              np.take_along_axis(near, k, 1), np.take_along_axis(band, k, 1)))
    # argmax over the GPU counts, ties to the lowest index
    bh = int(got["best_hyp"].reshape(-1)[0])
    bc = int(got["best_count"].reshape(-1)[0])
    if not valid_o.any():
        assert bh == -1 and bc == 0 and not got["mask"].any() and not got["best_H"].any()
        return ref
    assert bc == counts.max() and bh == int(np.argmax(counts == bc)), label
    if (lo[valid_o] == hi[valid_o]).all() and not borderline.any():
        assert bh == ref["best_hyp"] and bc == ref["best_count"], label
    # best H is the oracle's hypothesis bh (float64 ACA, pow2-scaled, rounded)
    Hg = got["best_H"].reshape(3, 3)
    assert hg.herr(Hg, ref["H32"][bh].astype(np.float64)) <= 1e-5, label
    # mask: the inliers of that H, outside the decision band
    d = oref.transfer_error(ref["H32"][bh:bh + 1], corr)[0]
    ex = np.abs(d - TAU) < BAND_PX
    m = got["mask"].astype(bool)
    assert np.array_equal(m[~ex], (d <= TAU)[~ex]), label
    assert int(m.sum()) == bc
    return ref


def run_single(corr_np, n_hyp, seed, plain=False, ld=None):
    import paper_2402_18008_amd as hgpu
    n = corr_np.shape[1]
    ld = n if ld is None else ld
    buf = torch.full((4, ld), float("nan"), device="cuda")
    buf[:, :n] = torch.from_numpy(corr_np)
    corr = buf[:, :n]
    fn = hgpu.hg_ransac_plain if plain else hgpu.hg_ransac
    out = fn(corr, n_hyp, TAU, seed)
    torch.cuda.synchronize()
    return to_np(out)


def test_config2_fused_and_plain():
    require_gpu()
    cs = synth.config2()
    announce("ransac fused config2 N=2000 hyps=4096")
    f = run_single(cs.corr, 4096, 2)
    announce("ransac plain config2")
    p = run_single(cs.corr, 4096, 2, plain=True)
    for k in f:
        assert np.array_equal(f[k], p[k]), k
    ref = check_pair(cs.corr, 4096, 2, f, label="config2")
    recall = (f["mask"].astype(bool) & cs.inlier).sum() / cs.inlier.sum()
    print("config2 best", int(f["best_count"][0]), "hyp", int(f["best_hyp"][0]), "recall", recall,
          "oracle best", ref["best_count"])
    assert recall > 0.6
    # run-to-run determinism
    g = run_single(cs.corr, 4096, 2)
    for k in f:
        assert np.array_equal(f[k], g[k]), k


@pytest.mark.parametrize("n,n_hyp,ld", [(4, 7, 4), (5, 100, 9), (33, 1000, 40), (257, 17, 300),
                                        (1500, 4097, 1500), (8000, 512, 8003)])
def test_sizes(n, n_hyp, ld):
    require_gpu()
    cs = synth.correspondences(n, 0.5, 1000 + n)
    announce(f"ransac n={n} hyps={n_hyp} ld={ld}")
    f = run_single(cs.corr, n_hyp, 77, ld=ld)
    p = run_single(cs.corr, n_hyp, 77, plain=True, ld=ld)
    for k in f:
        assert np.array_equal(f[k], p[k]), k
    check_pair(cs.corr, n_hyp, 77, f, label=f"n={n}")


def test_fused_matches_plain_over_sizes():
    """The fused form (8 waves per workgroup, hypotheses per workgroup chosen
    from the count) and the plain form (4 waves per workgroup) give identical
    outputs over pair sizes around every chunk boundary of either geometry and
    hypothesis counts that select every workgroup shape (both are the float64
    test's counts, so any difference is a geometry or tail error)."""
    require_gpu()
    rng = np.random.default_rng(20250)
    sizes = [4, 63, 64, 65, 511, 512, 513, 1023, 2047, 2049, 4095, 4096, 4097, 6000, 8191, 8193,
             12289, 20000]
    hyps = [1, 5, 63, 64, 1000, 2049, 4096, 9000, 16384, 40000]
    cases = [(int(n), int(rng.choice(hyps))) for n in sizes] + \
            [(int(rng.integers(4, 20000)), int(rng.integers(1, 40000))) for _ in range(6)]
    for k, (n, n_hyp) in enumerate(cases):
        cs = synth.correspondences(n, float(rng.uniform(0.2, 0.8)), 3000 + k)
        seed = int(rng.integers(0, 2**63))
        announce(f"ransac fused vs plain n={n} hyps={n_hyp} seed={seed}")
        f = run_single(cs.corr, n_hyp, seed)
        p = run_single(cs.corr, n_hyp, seed, plain=True)
        for key in f:
            assert np.array_equal(f[key], p[key]), (n, n_hyp, key)
        assert int(f["mask"].sum()) == int(f["best_count"][0]), (n, n_hyp)


def test_all_degenerate_and_nonfinite():
    require_gpu()
    corr = np.ones((4, 50), np.float32)
    announce("ransac all-degenerate")
    for plain in (False, True):
        f = run_single(corr, 64, 5, plain=plain)
        assert f["best_hyp"][0] == -1 and f["best_count"][0] == 0
        assert not f["mask"].any() and not f["best_H"].any() and not f["hyp_counts"].any()
    # a NaN point: samples containing it are invalid, it is never an inlier
    cs = synth.correspondences(300, 0.5, 9)
    corr = cs.corr.copy()
    corr[2, 5] = np.nan
    f = run_single(corr, 500, 3)
    check_pair(corr, 500, 3, f, label="nan")
    assert f["mask"][5] == 0


def test_seed_changes_samples():
    require_gpu()
    cs = synth.config2()
    a = run_single(cs.corr, 256, 1)
    b = run_single(cs.corr, 256, 2 | (1 << 40))
    assert not np.array_equal(a["hyp_counts"], b["hyp_counts"])
    check_pair(cs.corr, 256, 2 | (1 << 40), b, label="seed")


# ---- batched ----------------------------------------------------------------

_CONFIG3_REFS = []


def config3_refs():
    """Oracle references of the 512 config-3 pairs (1024 hypotheses, seed 3),
    computed once per session."""
    if not _CONFIG3_REFS:
        from tests.oracle_pool import ransac_refs
        cb = synth.config3()
        announce("oracle references of the 512 config-3 pairs (CPU process pool)")
        _CONFIG3_REFS.extend(ransac_refs(cb.corr, cb.off, 1024, TAU, 3))
    return _CONFIG3_REFS


def batched(cb, n_hyp=1024, seed=3, hyp_counts=True):
    import paper_2402_18008_amd as hgpu
    corr = torch.from_numpy(cb.corr).cuda()
    off = torch.from_numpy(cb.off).cuda()
    return hgpu.BatchedRansac(corr, off, n_hyp, TAU, seed, hyp_counts=hyp_counts)


def np_out(br):
    torch.cuda.synchronize()
    return dict(best_H=br.best_H.cpu().numpy(), best_count=br.best_count.cpu().numpy(),
                best_hyp=br.best_hyp.cpu().numpy(), mask=br.mask.cpu().numpy(),
                hyp_counts=br.hyp_counts.cpu().numpy())


def pair_view(cb, out, p):
    a, b = cb.off[p], cb.off[p + 1]
    return dict(best_H=out["best_H"][p], best_count=out["best_count"][p:p + 1],
                best_hyp=out["best_hyp"][p:p + 1], mask=out["mask"][a:b],
                hyp_counts=out["hyp_counts"][p])


def test_batched_small_all_tunings_identical():
    require_gpu()
    cb = synth.correspondence_batch(24, 31, n_min=4, n_max=3000)
    br = batched(cb, n_hyp=300, seed=11)
    ref = None
    for P in (8, 16):
        for HB in (16, 32, 64):
            for bpc in (1, 2, 4, 5, 6):
                announce(f"batched 24 pairs tuning P={P} HB={HB} bpc={bpc}")
                br.run((P, HB, bpc))
                out = np_out(br)
                if ref is None:
                    ref = out
                else:
                    for k in ref:
                        assert np.array_equal(ref[k], out[k]), (k, P, HB, bpc)
    for p in range(24):
        check_pair(cb.corr[:, cb.off[p]:cb.off[p + 1]], 300, 11, pair_view(cb, ref, p), pair=p,
                   label=f"pair {p}")


def test_config3_persistent_graph_and_autotune():
    require_gpu()
    cb = synth.config3()
    announce("batched config3 512 pairs x 1024 hyps: direct run")
    br = batched(cb)
    br.run()
    direct = np_out(br)
    # every pair against the oracle (references from a pool of CPU processes)
    refs = config3_refs()
    n_exempt = 0
    for p in range(512):
        check_pair(cb.corr[:, cb.off[p]:cb.off[p + 1]], 1024, 3, pair_view(cb, direct, p), pair=p,
                   label=f"config3 pair {p}", ref=refs[p])
        n_exempt += int(refs[p]["n_exempt"][refs[p]["valid"]].sum())
    print("config3: (hypothesis, point) pairs within 1e-4 px of the threshold:", n_exempt)
    announce("batched config3 autotune")
    tune = br.autotune(cb.off)
    print("autotuned", tune)
    br.run(tune)
    out = np_out(br)
    for k in direct:
        assert np.array_equal(direct[k], out[k]), k
    announce("batched config3 graph capture and replays")
    g = br.graph(tune)
    for rep in range(3):
        br.mask.zero_()
        br.best_count.fill_(-7)
        torch.cuda.synchronize()
        g.launch()
        out = np_out(br)
        for k in direct:
            assert np.array_equal(direct[k], out[k]), (k, rep)
    # change the buffer contents in place; the graph sees the new data
    perm = torch.from_numpy(np.random.default_rng(0).permutation(cb.corr.shape[1]))
    br.corr.copy_(br.corr[:, perm.cuda()].clone())
    torch.cuda.synchronize()
    g.launch()
    replay = np_out(br)
    br.run(tune)
    again = np_out(br)
    for k in replay:
        assert np.array_equal(replay[k], again[k]), k
    g.close()


def test_uncertified_and_overflowing_recount_list():
    """Exact inliers (x2 = x1 on an integer grid) scaled by 2^60: no point
    lies near the threshold, but for the hypotheses drawn from inliers the
    float32 certificate's magnitudes reach 1e18, so it certifies nothing and
    every group of theirs is listed for a float64 recount. A 64-hypothesis
    item of the batched kernel then lists more groups than the list holds and
    recounts every hypothesis of the item. Counts, best and masks equal the
    oracle's: single pair (fused, plain) and batched (two tunings)."""
    require_gpu()
    cb = synth.integer_identity_batch([5000, 3000, 700, 8000], 71, inlier_ratio=0.9)
    cb.corr *= np.float32(2.0 ** 60)
    from tests.oracle_pool import ransac_refs
    announce("oracle references of 4 scaled integer pairs")
    refs = ransac_refs(cb.corr, cb.off, 256, TAU, 5, workers=4)
    c0 = np.ascontiguousarray(cb.corr[:, cb.off[0]:cb.off[1]])
    for plain in (False, True):
        announce(f"ransac scaled integer pair 0 plain={plain}")
        got = run_single(c0, 256, 5, plain=plain)
        check_pair(c0, 256, 5, got, label=f"scaled pair 0 plain={plain}", ref=refs[0])
        assert int(got["best_count"][0]) == int(cb.inlier[cb.off[0]:cb.off[1]].sum())
    import paper_2402_18008_amd as hgpu
    br = hgpu.BatchedRansac(torch.from_numpy(cb.corr).cuda(), torch.from_numpy(cb.off).cuda(),
                            256, TAU, 5, hyp_counts=True)
    for tune in ((16, 64, 4), (8, 16, 2)):
        announce(f"batched scaled integer pairs tuning {tune}")
        br.run(tune)
        out = np_out(br)
        for p in range(4):
            check_pair(cb.corr[:, cb.off[p]:cb.off[p + 1]], 256, 5, pair_view(cb, out, p), pair=p,
                       label=f"scaled pair {p} tuning {tune}", ref=refs[p])


def test_outputs_without_hypothesis_counts():
    """Without the per-hypothesis count output the kernels recount in float64
    only the hypotheses that can still reach the best: best H, count, index
    and mask are those of the run with every count exact (single pair, plain
    and fused; the 512-pair batch)."""
    require_gpu()
    import paper_2402_18008_amd as hgpu
    from paper_2402_18008_amd import _abi
    cs = synth.config2()
    corr = torch.from_numpy(cs.corr).cuda()
    n, nh = corr.shape[1], 4096
    for name in ("hg_ransac", "hg_ransac_plain"):
        announce(f"{name} config2 with and without hyp_counts")
        outs = []
        for with_counts in (True, False):
            ws = torch.empty(hgpu.hg_ransac_ws_bytes(n, nh), dtype=torch.uint8, device="cuda")
            bh = torch.empty(9, device="cuda")
            bc = torch.empty(1, dtype=torch.int32, device="cuda")
            bi = torch.empty(1, dtype=torch.int32, device="cuda")
            mk = torch.empty(n, dtype=torch.uint8, device="cuda")
            hc = torch.empty(nh, dtype=torch.int32, device="cuda") if with_counts else None
            _abi.call(name, corr.data_ptr(), n, n, nh, TAU, 2, bh.data_ptr(), bc.data_ptr(),
                      bi.data_ptr(), mk.data_ptr(), hc.data_ptr() if with_counts else None,
                      ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
            torch.cuda.synchronize()
            outs.append([t.cpu().numpy() for t in (bh, bc, bi, mk)])
        for a, b in zip(*outs):
            assert np.array_equal(a, b), name
    cb = synth.config3()
    announce("batched config3 with and without hyp_counts")
    full = batched(cb, hyp_counts=True)
    full.run()
    fast = batched(cb, hyp_counts=False)
    fast.run()
    torch.cuda.synchronize()
    for k in ("best_H", "best_count", "best_hyp", "mask"):
        assert torch.equal(getattr(full, k), getattr(fast, k)), k


# ---- adaptive termination ------------------------------------------------------

def check_adaptive_pair(corr, n_hyp_max, seed, pair, got, label, full=None):
    """The GPU's stopping point lies between the sequential rule's stopping
    points with every exempt point an inlier and with every one an outlier
    (the rule is monotone in the best count), and equals it where those agree;
    the winner is the oracle's wherever no exempt point can change it."""
    ref = oref.ransac_adaptive_ref(corr, n_hyp_max, TAU, seed, pair=pair, band_px=BAND_PX,
                                   full=full)
    m_gpu = int(got["n_eval"])
    m_ref = ref["n_eval"]
    assert ref["n_eval_min"] <= m_gpu <= ref["n_eval_max"], (label, m_gpu, ref["n_eval_min"],
                                                              ref["n_eval_max"])
    if ref["n_eval_min"] == ref["n_eval_max"]:
        assert m_gpu == m_ref, (label, m_gpu, m_ref)
    valid, lo, hi = ref["valid"], ref["count_lo"], ref["count_hi"]
    exact = bool((lo[:m_gpu][valid[:m_gpu]] == hi[:m_gpu][valid[:m_gpu]]).all())
    assert m_gpu % 64 == 0 or m_gpu == n_hyp_max, label
    bh, bc = int(got["best_hyp"]), int(got["best_count"])
    v = valid[:m_gpu]
    if not v.any():
        assert bh == -1 and bc == 0 and not got["mask"].any()
        return ref
    assert 0 <= bh < m_gpu and valid[bh], label
    assert lo[bh] <= bc <= hi[bh], label
    assert bc >= lo[:m_gpu][v].max(), label
    if exact and m_gpu == m_ref:
        assert bh == ref["best_hyp"] and bc == ref["best_count"], label
    Hg = got["best_H"].reshape(3, 3)
    assert hg.herr(Hg, ref["H32"][bh].astype(np.float64)) <= 1e-5, label
    d = oref.transfer_error(ref["H32"][bh:bh + 1], corr)[0]
    ex = np.abs(d - TAU) < BAND_PX
    mk = got["mask"].astype(bool)
    assert np.array_equal(mk[~ex], (d <= TAU)[~ex]), label
    assert int(mk.sum()) == bc
    return ref


def test_adaptive_termination_against_oracle():
    require_gpu()
    import paper_2402_18008_amd as hgpu
    cb = synth.correspondence_batch(40, 41, n_min=60, n_max=3000)
    corr = torch.from_numpy(cb.corr).cuda()
    off = torch.from_numpy(cb.off).cuda()
    ar = hgpu.AdaptiveRansac(corr, off, 1000, TAU, 17, confidence=0.99)
    ref = None
    for tune in ((8, 64, 1), (8, 64, 4), (16, 64, 2), (16, 64, 8), None):
        announce(f"adaptive 40 pairs tuning {tune}")
        ar.run(tune)
        torch.cuda.synchronize()
        out = dict(best_H=ar.best_H.cpu().numpy(), best_count=ar.best_count.cpu().numpy(),
                   best_hyp=ar.best_hyp.cpu().numpy(), n_eval=ar.n_evaluated.cpu().numpy(),
                   mask=ar.mask.cpu().numpy())
        if ref is None:
            ref = out
        else:
            for k in ref:
                assert np.array_equal(ref[k], out[k]), (k, tune)
    evals = []
    for p in range(40):
        a, b = cb.off[p], cb.off[p + 1]
        got = dict(best_H=ref["best_H"][p], best_count=ref["best_count"][p],
                   best_hyp=ref["best_hyp"][p], n_eval=ref["n_eval"][p], mask=ref["mask"][a:b])
        check_adaptive_pair(cb.corr[:, a:b], 1000, 17, p, got, f"adaptive pair {p}")
        evals.append(int(ref["n_eval"][p]))
    print("adaptive n_evaluated", evals)
    assert min(evals) < 1000 and max(evals) <= 1000


def test_adaptive_extremes():
    require_gpu()
    import paper_2402_18008_amd as hgpu
    sets = [synth.correspondences(500, 0.95, 51), synth.correspondences(500, 0.05, 52),
            synth.correspondences(4, 1.0, 53)]
    corr = np.concatenate([s.corr for s in sets], axis=1)
    off = np.array([0, 500, 1000, 1004], np.int64)
    ar = hgpu.AdaptiveRansac(torch.from_numpy(corr).cuda(), torch.from_numpy(off).cuda(), 700, TAU, 3)
    announce("adaptive extremes")
    ar.run()
    torch.cuda.synchronize()
    ne = ar.n_evaluated.cpu().numpy()
    assert ne[0] == 64            # 95 % inliers: one round is enough
    assert ne[1] == 700           # 5 % inliers: the cap
    for p in range(3):
        a, b = off[p], off[p + 1]
        got = dict(best_H=ar.best_H[p].cpu().numpy(), best_count=int(ar.best_count[p]),
                   best_hyp=int(ar.best_hyp[p]), n_eval=int(ne[p]), mask=ar.mask[a:b].cpu().numpy())
        check_adaptive_pair(corr[:, a:b], 700, 3, p, got, f"extreme {p}")


def test_adaptive_equal_and_odd_ratio_sizes():
    """Pairs of 300, 900 and 1500 points (equal sizes, and size ratios 3 and 5,
    give rounds with equal queue keys): every pair finishes, at the oracle's
    stopping round, with the oracle's result, for two tunings alike."""
    require_gpu()
    import paper_2402_18008_amd as hgpu
    sizes = [300, 900, 1500, 300, 300, 900, 1500, 1500, 900, 300, 300, 900]
    ratios = [0.25, 0.5, 0.3, 0.9, 0.2, 0.35, 0.6, 0.22, 0.8, 0.4, 0.3, 0.25]
    sets = [synth.correspondences(n, r, 200 + i) for i, (n, r) in enumerate(zip(sizes, ratios))]
    corr = np.ascontiguousarray(np.concatenate([s.corr for s in sets], axis=1))
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    ar = hgpu.AdaptiveRansac(torch.from_numpy(corr).cuda(), torch.from_numpy(off).cuda(), 1000,
                             TAU, 29, confidence=0.99)
    ref = None
    for tune in ((16, 64, 4), (8, 64, 1)):
        announce(f"adaptive equal/odd-ratio sizes tuning {tune}")
        ar.run(tune)
        torch.cuda.synchronize()
        out = dict(best_H=ar.best_H.cpu().numpy(), best_count=ar.best_count.cpu().numpy(),
                   best_hyp=ar.best_hyp.cpu().numpy(), n_eval=ar.n_evaluated.cpu().numpy(),
                   mask=ar.mask.cpu().numpy())
        if ref is None:
            ref = out
        else:
            for k in ref:
                assert np.array_equal(ref[k], out[k]), (k, tune)
    for p in range(len(sizes)):
        a, b = off[p], off[p + 1]
        got = dict(best_H=ref["best_H"][p], best_count=ref["best_count"][p],
                   best_hyp=ref["best_hyp"][p], n_eval=ref["n_eval"][p], mask=ref["mask"][a:b])
        check_adaptive_pair(corr[:, a:b], 1000, 29, p, got, f"equal-size pair {p}")


def test_adaptive_config3_all_pairs():
    """Adaptive termination on the 512-pair workload in the benchmark's launch
    shape (16 points per lane, 4 workgroups per CU): every pair against the
    oracle's sequential rule. Two other shapes (8 points per lane at 6
    workgroups per CU, and the library's own choice) give identical outputs."""
    require_gpu()
    import paper_2402_18008_amd as hgpu
    cb = synth.config3()
    ar = hgpu.AdaptiveRansac(torch.from_numpy(cb.corr).cuda(), torch.from_numpy(cb.off).cuda(),
                             1024, TAU, 3, confidence=0.99)
    out = None
    for tune in ((16, 64, 4), (8, 64, 6), None):
        announce(f"adaptive config3 512 pairs, cap 1024, tuning {tune}")
        ar.run(tune)
        torch.cuda.synchronize()
        got = dict(best_H=ar.best_H.cpu().numpy(), best_count=ar.best_count.cpu().numpy(),
                   best_hyp=ar.best_hyp.cpu().numpy(), n_eval=ar.n_evaluated.cpu().numpy(),
                   mask=ar.mask.cpu().numpy())
        if out is None:
            out = got
        else:
            for k in out:
                assert np.array_equal(out[k], got[k]), (k, tune)
    ne = out["n_eval"]
    assert np.all((ne % 64 == 0) | (ne == 1024)) and ne.min() >= 64 and ne.max() <= 1024
    for p in range(512):
        a, b = cb.off[p], cb.off[p + 1]
        assert int(out["mask"][a:b].sum()) == int(out["best_count"][p]), p
    refs = config3_refs()
    for p in range(512):
        a, b = cb.off[p], cb.off[p + 1]
        got = dict(best_H=out["best_H"][p], best_count=out["best_count"][p],
                   best_hyp=out["best_hyp"][p], n_eval=ne[p], mask=out["mask"][a:b])
        check_adaptive_pair(cb.corr[:, a:b], 1024, 3, p, got, f"adaptive config3 pair {p}",
                            full=refs[p])


def test_batched_rejects_bad_offsets():
    """Offsets are checked on the host before any launch: decreasing, out of
    range, or a pair with fewer than 4 points is refused."""
    require_gpu()
    import paper_2402_18008_amd as hgpu
    corr = torch.zeros((4, 100), device="cuda")
    for bad in ([0, 50, 40, 100], [0, 50, 101], [-1, 50, 100], [0, 3, 100]):
        off = torch.tensor(bad, dtype=torch.int64, device="cuda")
        with pytest.raises(ValueError):
            hgpu.BatchedRansac(corr, off, 64, TAU, 1)
        with pytest.raises(ValueError):
            hgpu.AdaptiveRansac(corr, off, 64, TAU, 1)
    off = torch.tensor([0, 50, 100], dtype=torch.int64, device="cuda")
    with pytest.raises(ValueError):
        hgpu.hg_refit_ho(corr, off, H=torch.empty(9, device="cuda"))
