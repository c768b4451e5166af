"""Workload generators: determinism, shapes and the stated distributions."""
import numpy as np

import synth


def test_quadruples_deterministic_and_chunked():
    a = synth.quadruples(3000, 5)
    b = synth.quadruples(3000, 5)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    src, dst, lab = a
    assert src.shape == (8, 3000) and src.dtype == np.float32 and not lab.any()
    assert (src[0::2] >= 0).all() and (src[0::2] <= 640).all()
    assert (src[1::2] >= 0).all() and (src[1::2] <= 480).all()


def test_quadruples_parallel_equals_serial(monkeypatch):
    monkeypatch.setattr(synth, "CHUNK", 1000)
    s1 = synth.quadruples(3500, 9, degenerate_every=100)
    s2 = synth.quadruples_parallel(3500, 9, degenerate_every=100, workers=3)
    for x, y in zip(s1, s2):
        assert np.array_equal(x, y)
    assert s1[2].sum() == 35


def test_correspondence_sets():
    cs = synth.config2()
    assert cs.corr.shape == (4, 2000) and cs.inlier.sum() == 600
    b = synth.correspondence_batch(20, 3)
    ns = np.diff(b.off)
    assert (ns >= 100).all() and (ns <= 8000).all()
    assert b.corr.shape == (4, b.off[-1])
    assert np.array_equal(b.corr, synth.correspondence_batch(20, 3).corr)


def test_patches():
    pb = synth.patches(4, 4)
    assert pb.img.shape == (4, 128, 128) and pb.tgt.shape == (4, 128, 128)
    assert np.allclose(pb.img.mean(axis=(1, 2)), 0, atol=1e-5)
    assert np.allclose(pb.img.std(axis=(1, 2)), 1, atol=1e-4)
    assert (np.abs(pb.offsets) <= 32).all()


def test_pattern_images():
    d1 = synth.pattern_images(1000, 4)
    d2 = synth.pattern_images(1000, 4, workers=2)
    assert d1.shape == (8, 1000) and d1.dtype == np.float32
    assert np.array_equal(d1, d2)
    assert not np.array_equal(d1, synth.pattern_images(1000, 5))
    # the pattern's centroid lands near the frame centre; sizes follow the scale draw
    cx = d1[0::2].mean(axis=0)
    cy = d1[1::2].mean(axis=0)
    assert abs(np.median(cx) - 320) < 15 and abs(np.median(cy) - 240) < 15
    span = np.hypot(d1[2] - d1[0], d1[3] - d1[1])          # image of the M N edge (160 units)
    assert 0.4 * 160 < np.median(span) < 2.5 * 160


# ---- distributions of the drawn parameters (KS / chi-square pins) ------------

from scipy import stats  # noqa: E402

P_MIN = 1e-4   # fixed seeds: each statistic is a fixed number; this is far below typical p-values


def _uniform_p(x, lo, hi):
    return stats.kstest(np.asarray(x, np.float64), "uniform", args=(lo, hi - lo)).pvalue


def _similarity_params(H):
    s = np.hypot(H[:, 0, 0], H[:, 1, 0])
    th = np.arctan2(H[:, 1, 0], H[:, 0, 0])
    return s, th, H[:, 0, 2], H[:, 1, 2], H[:, 2, 0], H[:, 2, 1]


def test_similarity_perspective_draws():
    """Scale U[0.5, 2], rotation U[-pi, pi], translation U[-100, 100]^2,
    perspective U[-1e-3, 1e-3]^2, h33 = 1, and the rotation block orthogonal."""
    H = synth._random_similarity_persp(np.random.default_rng(123), 100000)
    s, th, tx, ty, p, q = _similarity_params(H)
    assert np.allclose(H[:, 0, 0], H[:, 1, 1]) and np.allclose(H[:, 0, 1], -H[:, 1, 0])
    assert np.all(H[:, 2, 2] == 1.0)
    for x, lo, hi in ((s, 0.5, 2.0), (th, -np.pi, np.pi), (tx, -100, 100), (ty, -100, 100),
                      (p, -1e-3, 1e-3), (q, -1e-3, 1e-3)):
        assert x.min() >= lo and x.max() <= hi
        assert _uniform_p(x, lo, hi) > P_MIN


def test_quadruple_chunk_distributions():
    """Source points uniform in the frame; every point has w >= 0.1 after the
    perspective redraw (which changes few draws); target noise N(0, 0.5^2);
    planted near-degenerate sets have a triangle of height <= 1e-3 px."""
    src, dst, lab, H = synth.quadruple_chunk(1, 0, degenerate_every=100, m=50000, with_h=True)
    s, th, tx, ty, p, q = _similarity_params(H)
    for x, lo, hi in ((s, 0.5, 2.0), (th, -np.pi, np.pi), (tx, -100, 100)):
        assert _uniform_p(x, lo, hi) > P_MIN
    ok = lab == 0
    assert _uniform_p(src[0::2][:, ok].ravel(), 0, 640) > P_MIN
    assert _uniform_p(src[1::2][:, ok].ravel(), 0, 480) > P_MIN
    x, y = src[0::2].astype(np.float64), src[1::2].astype(np.float64)
    w = H[:, 2, 0, None] * x.T + H[:, 2, 1, None] * y.T + 1.0
    assert w.min() >= 0.1
    # the redraw only trims the corner of the perspective square that folds the frame
    assert abs(np.mean(p < 0) - 0.5) < 0.02 and np.abs(p).max() <= 1e-3
    u = H[:, 0, 0, None] * x.T + H[:, 0, 1, None] * y.T + H[:, 0, 2, None]
    v = H[:, 1, 0, None] * x.T + H[:, 1, 1, None] * y.T + H[:, 1, 2, None]
    nx = dst[0::2].T[ok] - (u / w)[ok]
    ny = dst[1::2].T[ok] - (v / w)[ok]
    for r in (nx.ravel(), ny.ravel()):
        assert stats.kstest(r[:40000], "norm", args=(0.0, 0.5)).pvalue > P_MIN
    # planted sets: some triangle of the source side is within 1e-3 px of a line
    assert np.array_equal(np.nonzero(lab)[0], np.arange(0, 50000, 100))
    pts = np.stack([x, y], axis=-1)[:, lab == 1]          # (4, k, 2)
    hmin = np.full(pts.shape[1], np.inf)
    for a, b, c in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)):
        for i, j, k in ((a, b, c), (b, c, a), (c, a, b)):
            e = pts[j] - pts[i]
            f = pts[k] - pts[i]
            area = np.abs(e[:, 0] * f[:, 1] - e[:, 1] * f[:, 0])
            hmin = np.minimum(hmin, area / np.hypot(e[:, 0], e[:, 1]))
    assert hmin.max() <= 1e-3 + 1e-3         # 1e-3 px planted, plus float32 rounding of the points


def _centred(H):
    T = np.array([[1.0, 0, 320], [0, 1, 240], [0, 0, 1]])
    Ti = np.array([[1.0, 0, -320], [0, 1, -240], [0, 0, 1]])
    return Ti @ H @ T


def test_correspondence_batch_distributions():
    """Config-3 pairs: N_p ~ U{100..8000}, inlier ratio U[0.1, 0.9] with
    round(ratio N) inliers; ground-truth H drawn as for the quadruples and
    conjugated to act about the frame centre; inlier noise N(0, 1) px;
    outliers uniform on both sides."""
    b = synth.config3()
    ns = np.diff(b.off)
    assert ns.min() >= 100 and ns.max() <= 8000
    # discrete uniform on {100..8000}: KS against the continuous law of N + U[0, 1)
    jitter = np.random.default_rng(0).uniform(0, 1, ns.size)
    assert _uniform_p(ns + jitter, 100, 8001) > P_MIN
    assert _uniform_p(b.ratio, 0.1, 0.9) > P_MIN
    n_in = np.add.reduceat(b.inlier.astype(np.int64), b.off[:-1])
    assert np.array_equal(n_in, np.round(b.ratio * ns).astype(np.int64))
    H = np.stack([_centred(h) for h in b.H_true])
    s, th, tx, ty, p, q = _similarity_params(H)
    for x, lo, hi in ((s, 0.5, 2.0), (th, -np.pi, np.pi), (tx, -100, 100), (p, -1e-3, 1e-3)):
        assert _uniform_p(x, lo, hi) > P_MIN
    # inlier residuals and outlier positions, over the first 64 pairs
    res, outx = [], []
    for k in range(64):
        a, e = b.off[k], b.off[k + 1]
        c = b.corr[:, a:e].astype(np.float64)
        m = b.inlier[a:e]
        Hk = b.H_true[k]
        w = Hk[2, 0] * c[0] + Hk[2, 1] * c[1] + Hk[2, 2]
        u = (Hk[0, 0] * c[0] + Hk[0, 1] * c[1] + Hk[0, 2]) / w
        v = (Hk[1, 0] * c[0] + Hk[1, 1] * c[1] + Hk[1, 2]) / w
        res += [(c[2] - u)[m], (c[3] - v)[m]]
        outx.append(c[2][~m])
    r = np.concatenate(res)
    assert stats.kstest(r, "norm", args=(0.0, 1.0)).pvalue > P_MIN
    assert _uniform_p(np.concatenate(outx), 0, 640) > P_MIN


def test_patch_offsets_and_shifts():
    pb = synth.patches(1024, 4, size=8)
    assert _uniform_p(pb.offsets.ravel(), -32, 32) > P_MIN
    counts = np.bincount((pb.shift + 16).ravel(), minlength=33)
    assert counts.size == 33 and stats.chisquare(counts).pvalue > P_MIN


def test_integer_identity_batch():
    """Exact-inlier pairs: integer coordinates in range, x2 = x1 exactly on the
    inliers and never on the outliers, the requested inlier fraction, and the
    same draw for the same seed."""
    cb = synth.integer_identity_batch([500, 37, 2000], 5, inlier_ratio=0.7, side=16)
    assert cb.corr.dtype == np.float32 and cb.off.tolist() == [0, 500, 537, 2537]
    c = cb.corr.astype(np.float64)
    assert (c == np.round(c)).all() and c.min() >= 0 and c.max() <= 15
    same = (c[:2] == c[2:]).all(axis=0)
    assert np.array_equal(same, cb.inlier)
    assert abs(cb.inlier.mean() - 0.7) < 0.05
    again = synth.integer_identity_batch([500, 37, 2000], 5, inlier_ratio=0.7, side=16)
    assert np.array_equal(again.corr, cb.corr)
