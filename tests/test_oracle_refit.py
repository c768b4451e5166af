"""Pins for the oracle's HO-SVD refit (CPU only).

The refit is checked against exact data (it must return the homography that
generated noise-free points, and the exact DLT on 4 points), against its
defining property on noisy data (no nearby homography, and no result of a
general-purpose minimiser, has a smaller HO objective), and against the
similarity invariance that the normalisation gives it."""
from fractions import Fraction

import numpy as np
from scipy import optimize

import synth
from oracle import homography as hg
from oracle import refit


def project(H, x, y):
    w = H[2, 0] * x + H[2, 1] * y + H[2, 2]
    return (H[0, 0] * x + H[0, 1] * y + H[0, 2]) / w, (H[1, 0] * x + H[1, 1] * y + H[1, 2]) / w


def random_h(rng):
    cs = synth.correspondences(10, 0.5, int(rng.integers(1 << 30)))
    return cs.H_true


def test_exact_data_is_recovered():
    rng = np.random.default_rng(0)
    for n in (4, 5, 10, 1000):
        H = random_h(rng)
        x = rng.uniform(0, 640, n)
        y = rng.uniform(0, 480, n)
        u, v = project(H, x, y)
        assert hg.herr(refit.ho_svd(x, y, u, v), H) < 1e-10, n


def test_four_points_equal_exact_dlt():
    rng = np.random.default_rng(1)
    for _ in range(50):
        s = [Fraction(int(a)) for a in rng.integers(0, 100, 8)]
        d = [Fraction(int(a)) for a in rng.integers(0, 100, 8)]
        try:
            Hx = hg.exact_h(s, d)
        except ZeroDivisionError:
            continue
        f = [float(a) for a in s + d]
        H = refit.ho_svd(f[0:8:2], f[1:8:2], f[8:16:2], f[9:16:2])
        assert hg.herr(H, Hx) < 1e-9


def test_minimises_the_ho_objective():
    """On noisy inliers no homography near the result, and none found by a
    general-purpose minimiser started at the normalised DLT, has a smaller
    ||A h|| / ||h3|| in normalised coordinates."""
    rng = np.random.default_rng(2)
    for trial in range(5):
        cs = synth.correspondences(300, 1.0, 100 + trial)
        x1, y1, x2, y2 = (cs.corr[k].astype(np.float64) for k in range(4))
        H = refit.ho_svd(x1, y1, x2, y2)
        f0 = refit.algebraic_residual(H, x1, y1, x2, y2)
        for _ in range(50):
            Hp = H * (1 + 1e-4 * rng.normal(size=(3, 3)))
            assert refit.algebraic_residual(Hp, x1, y1, x2, y2) >= f0
        h0 = H.ravel() / H[2, 2]

        def obj(p):
            return refit.algebraic_residual(np.append(p, 1.0).reshape(3, 3), x1, y1, x2, y2)

        res = optimize.minimize(obj, h0[:8] * (1 + 1e-3 * rng.normal(size=8)), method="Nelder-Mead",
                                options=dict(xatol=1e-12, fatol=1e-14, maxiter=20000, maxfev=40000))
        assert res.fun >= f0 * (1 - 1e-9)
        # and the noise-free homography is close (1 px noise, 300 inliers)
        assert hg.herr(H, cs.H_true) < 1e-2


def test_similarity_invariance_and_order():
    rng = np.random.default_rng(3)
    cs = synth.correspondences(200, 1.0, 7)
    x1, y1, x2, y2 = (cs.corr[k].astype(np.float64) for k in range(4))
    H = refit.ho_svd(x1, y1, x2, y2)
    th, sc = 0.7, 1.9
    S = np.array([[sc * np.cos(th), -sc * np.sin(th), 30.0], [sc * np.sin(th), sc * np.cos(th), -12.0],
                  [0.0, 0.0, 1.0]])
    xs, ys = project(S, x1, y1)
    Hs = refit.ho_svd(xs, ys, x2, y2)
    assert hg.herr(Hs, H @ np.linalg.inv(S)) < 1e-9
    perm = rng.permutation(200)
    assert hg.herr(refit.ho_svd(x1[perm], y1[perm], x2[perm], y2[perm]), H) < 1e-12


def test_refit_ref_masks():
    b = synth.correspondence_batch(6, 9, n_min=100, n_max=400)
    mask = b.inlier.astype(np.uint8).copy()
    mask[b.off[2]:b.off[3]] = 0
    mask[b.off[3]:b.off[3] + 3] = 1
    mask[b.off[3] + 3:b.off[4]] = 0
    H, used = refit.refit_ref(b.corr, b.off, mask)
    assert used[2] == 0 and used[3] == 3 and not H[2].any() and not H[3].any()
    for p in (0, 1, 4, 5):
        a, e = b.off[p], b.off[p + 1]
        sel = np.nonzero(mask[a:e])[0] + a
        Hp = refit.ho_svd(*(b.corr[k, sel] for k in range(4)))
        assert np.array_equal(H[p], Hp) and used[p] == sel.size
        assert hg.herr(H[p], b.H_true[p]) < 2e-2
