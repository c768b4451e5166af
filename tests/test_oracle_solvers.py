"""Pins for the oracle's 4-point solvers (CPU only).

Each oracle solver is checked against something other than itself: the exact
rational DLT (the plain definition x2 ~ H x1), the paper's invariants
(Propositions 1 and 4, canonical anchor points), special cases (affine input,
rectangle source), a library routine (SVD null vector) and the paper's FLOP
tables.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import homography as hg
from oracle import flops


def rand_int_quads(rng, k, lo=0, hi=100):
    return [[Fraction(int(v)) for v in rng.integers(lo, hi, 8)] for _ in range(k)], \
           [[Fraction(int(v)) for v in rng.integers(lo, hi, 8)] for _ in range(k)]


def cross_zero(H, src, dst):
    """x2 x (H x1) == 0 for all four correspondences (exact)."""
    for k in range(4):
        u, v, w = hg.apply3(H, src[2 * k], src[2 * k + 1])
        x, y = dst[2 * k], dst[2 * k + 1]
        if (y * w - v, u - x * w, x * v - y * u) != (0, 0, 0):
            return False
    return True


def proportional(A, B):
    a = [x for r in A for x in r]
    b = [x for r in B for x in r]
    k = next(i for i in range(9) if b[i] != 0)
    lam = a[k] / b[k]
    return lam != 0 and all(a[i] == lam * b[i] for i in range(9))


def generic(src, dst):
    try:
        hg.dlt_s(src, dst)
    except ZeroDivisionError:
        return False
    X = [src[0::2], dst[0::2]]
    Y = [src[1::2], dst[1::2]]
    for s in range(2):
        for a, b, c in itertools.combinations(range(4), 3):
            if (X[s][b] - X[s][a]) * (Y[s][c] - Y[s][a]) - (Y[s][b] - Y[s][a]) * (X[s][c] - X[s][a]) == 0:
                return False
    return True


@pytest.fixture(scope="module")
def int_quads():
    rng = np.random.default_rng(123)
    S, D = rand_int_quads(rng, 260)
    pairs = [(s, d) for s, d in zip(S, D) if generic(s, d)]
    assert len(pairs) >= 200
    return pairs[:200]


def test_dlt_exact_satisfies_definition(int_quads):
    for s, d in int_quads:
        H = hg.dlt_s(s, d)
        assert cross_zero(H, s, d)


def test_dlt64_matches_svd_null_vector():
    src, dst, _ = synth.quadruples(256, 7)
    H = hg.dlt64(src, dst)
    s = src.astype(np.float64)
    d = dst.astype(np.float64)
    for i in range(0, 256, 8):
        A = []
        for k in range(4):
            x, y, u, v = s[2 * k, i], s[2 * k + 1, i], d[2 * k, i], d[2 * k + 1, i]
            A.append([x, y, 1, 0, 0, 0, -u * x, -u * y, -u])
            A.append([0, 0, 0, x, y, 1, -v * x, -v * y, -v])
        # scale columns so the SVD works on a balanced matrix, then undo
        A = np.array(A)
        cs = np.abs(A).max(axis=0)
        _, _, Vt = np.linalg.svd(A / cs)
        h = Vt[-1] / cs
        assert hg.herr(H[i], h.reshape(3, 3)) < 1e-7


def test_aca_proportional_to_exact_dlt(int_quads):
    for s, d in int_quads:
        assert proportional(hg.aca_s(s, d), hg.dlt_s(s, d))


def test_aca_structured_equals_matrix_product(int_quads):
    for s, d in int_quads[:100]:
        assert hg.aca_s(s, d) == hg.aca_matrix_s(s, d)


def test_aca_polynomial_form(int_quads):
    for s, d in int_quads[:100]:
        assert hg.aca_poly_s(s, d) == hg.aca_s(s, d)
    # the third column as typeset (f_A1) does not give the homography
    bad = sum(not proportional(hg.aca_poly_s(s, d, printed=True), hg.dlt_s(s, d))
              for s, d in int_quads[:50])
    assert bad == 50
    # smallest example: a unit square onto itself must give a multiple of I
    sq = [Fraction(v) for v in (1, 1, 2, 1, 1, 2, 2, 2)]
    Hc = hg.aca_poly_s(sq, sq)
    assert proportional(Hc, [[1, 0, 0], [0, 1, 0], [0, 0, 1]])
    Hp = hg.aca_poly_s(sq, sq, printed=True)
    assert not proportional(Hp, [[1, 0, 0], [0, 1, 0], [0, 0, 1]])


def test_aca_polynomial_degrees():
    # degrees 8 8 7 / 8 8 9 ... as stated: scale all 16 inputs by k, h_ij scales by k^deg
    rng = np.random.default_rng(5)
    s = [Fraction(int(v)) for v in rng.integers(1, 50, 8)]
    d = [Fraction(int(v)) for v in rng.integers(1, 50, 8)]
    H1 = hg.aca_poly_s(s, d)
    k = Fraction(3)
    H3 = hg.aca_poly_s([k * v for v in s], [k * v for v in d])
    deg = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            # homogeneous polynomials: h(k x) = k^deg h(x)
            r = H3[i][j] / H1[i][j]
            e = 0
            while r > 1:
                r /= 3
                e += 1
            assert r == 1
            deg[i][j] = e
    assert deg == [[8, 8, 9], [8, 8, 9], [7, 7, 8]]


def test_aca_invariants(int_quads):
    canon = [(0, 0), (1, 0), (0, 1)]
    for s, d in int_quads[:60]:
        HA1, HA2, HA2inv, HC = hg.aca_parts_s(s, d)
        for side, Hs in ((s, HA1), (d, HA2)):
            for k in range(3):
                u, v, w = hg.apply3(Hs, side[2 * k], side[2 * k + 1])
                assert (u / w, v / w) == canon[k]
        # the closed-form inverses (eq. inverseAffineOfA1) invert H_A up to scale
        HA1inv = hg.aca_parts_s(d, s)[2]
        eye = [[1, 0, 0], [0, 1, 0], [0, 0, 1]]
        assert proportional(hg.matmul3(HA1, HA1inv), eye)
        assert proportional(hg.matmul3(HA2, HA2inv), eye)
        # Proposition 4: the core fixes the three canonical anchor points
        for x, y in canon:
            u, v, w = hg.apply3(HC, Fraction(x), Fraction(y))
            assert w != 0 and (u / w, v / w) == (x, y)
        # Q3 = H_A1 Q1 has (Q3.x, Q3.y, f_A1) = doubled signed areas of MQP, MNQ, MNP,
        # and t1 = f_A1 - Q3.x - Q3.y that of NPQ
        M, N, P, Q = [(s[2 * k], s[2 * k + 1]) for k in range(4)]
        cr = lambda a, b, c: (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
        Q3 = hg.apply3(HA1, Q[0], Q[1])
        assert Q3 == (cr(M, Q, P), cr(M, N, Q), cr(M, N, P))
        assert Q3[2] - Q3[0] - Q3[1] == cr(N, P, Q)


def test_sks_proportional_to_exact_dlt(int_quads):
    n = 0
    for s, d in int_quads:
        try:
            H = hg.sks_s(s, d)
        except ZeroDivisionError:
            continue          # a + b or a - b denominator vanishes (measure zero)
        assert proportional(H, hg.dlt_s(s, d))
        n += 1
    assert n >= 190


def test_sks_invariants(int_quads):
    for s, d in int_quads[:60]:
        try:
            HS1, HS2, HS2inv, HK, H = hg.sks_parts_s(s, d)
        except ZeroDivisionError:
            continue
        for side, Hs in ((s, HS1), (d, HS2)):
            for k, target in ((0, (-1, 0)), (1, (1, 0))):
                u, v, w = hg.apply3(Hs, side[2 * k], side[2 * k + 1])
                assert (u / w, v / w) == target
        # Proposition 1: H_K fixes (-1, 0) and (1, 0) and has the structure [[a,u,b],[0,1,0],[b,v,a]]
        for x in (-1, 1):
            u, v, w = hg.apply3(HK, Fraction(x), Fraction(0))
            assert (u / w, v / w) == (x, 0)
        assert HK[0][0] == HK[2][2] and HK[0][2] == HK[2][0] and HK[1] == [0, 1, 0]
        # the composition is the same homography
        assert proportional(hg.matmul3(hg.matmul3(HS2inv, HK), HS1), H)


def test_sk_simplified_exact(int_quads):
    """Simplified SK (eq. SK): Hbar H_S1 is the homography through the four
    correspondences, H_S1 takes the pattern's anchors to (-1, 0), (1, 0), and
    Hbar takes those canonical anchors to the image's anchors (exact)."""
    n = 0
    for s, d in int_quads:
        try:
            pat = hg.sk_pattern_s(s)
            Hb = hg.sk_simplified_s(pat, d)
        except ZeroDivisionError:
            continue          # a Q7 denominator of the pattern vanishes
        HS1 = pat[4]
        assert proportional(hg.matmul3(Hb, HS1), hg.dlt_s(s, d))
        for k, x in ((0, -1), (1, 1)):
            u, v, w = hg.apply3(HS1, s[2 * k], s[2 * k + 1])
            assert (u / w, v / w) == (x, 0)
            u, v, w = hg.apply3(Hb, Fraction(x), Fraction(0))
            assert (u / w, v / w) == (d[2 * k], d[2 * k + 1])
        n += 1
    assert n >= 190
    # a pattern already in its canonical frame: H_S1 is a multiple of I and
    # Hbar is the homography itself
    obj = [Fraction(v) for v in (-1, 0, 1, 0, 3, 7, -2, 5)]
    d = [Fraction(v) for v in (10, 12, 61, 8, 14, 47, 55, 52)]
    pat = hg.sk_pattern_s(obj)
    assert proportional(pat[4], [[1, 0, 0], [0, 1, 0], [0, 0, 1]])
    assert proportional(hg.sk_simplified_s(pat, d), hg.dlt_s(obj, d))


def test_affine_normalised_exact():
    """Three correspondences of a known integer affine map give back exactly
    that map (the 2 x 3 [A | t] with x' = A x + t)."""
    rng = np.random.default_rng(12)
    n = 0
    for _ in range(100):
        A = [[Fraction(int(v)) for v in rng.integers(-5, 6, 3)] for _ in range(2)]
        src = [Fraction(int(v)) for v in rng.integers(-20, 20, 6)]
        (x0, y0), (x1, y1), (x2, y2) = src[0:2], src[2:4], src[4:6]
        if (x1 - x0) * (y2 - y0) - (y1 - y0) * (x2 - x0) == 0:
            continue
        dst = []
        for k in range(3):
            x, y = src[2 * k], src[2 * k + 1]
            dst += [A[0][0] * x + A[0][1] * y + A[0][2], A[1][0] * x + A[1][1] * y + A[1][2]]
        assert hg.affine_normalised_s(src, dst) == A
        n += 1
    assert n >= 90


def test_affine_and_sk_flags():
    # exactly collinear triangle on either side, a NaN; flags of a generic set clear
    src, dst, _ = synth.quadruples(4, 3)
    src[:, 0] = [0, 0, 10, 10, 20, 20, 5, 40]
    dst[:6, 1] = [1, 1, 2, 2, 3, 3]
    src[3, 2] = np.nan
    f = hg.affine_flags(src[:6], dst[:6])
    assert list(f) == [1, 1, 2, 0]
    obj = [0.0, 0.0, 100.0, 0.0, 0.0, 80.0, 120.0, 90.0]
    g = hg.sk_flags(obj, dst)
    assert g[1] == 1 and g[0] == 0 and g[3] == 0
    # a pattern with three collinear points flags every image
    assert (hg.sk_flags([0, 0, 100, 0, 50, 0, 120, 90], dst[:, 2:]) == 1).all()


def test_rect_algorithm1(int_quads):
    rng = np.random.default_rng(9)
    for _ in range(100):
        x0, y0 = Fraction(int(rng.integers(-50, 50))), Fraction(int(rng.integers(-50, 50)))
        w = Fraction(int(rng.integers(1, 60)))
        hgt = Fraction(int(rng.integers(1, 60)))
        r = w / hgt
        src = hg.rect_corners(x0, y0, w, r)
        dst = [Fraction(int(v)) for v in rng.integers(-100, 200, 8)]
        if not generic(src, dst):
            continue
        assert proportional(hg.aca_rect_s(x0, y0, w, r, dst), hg.aca_s(src, dst))
        if r == 1:
            assert hg.aca_rect_s(x0, y0, w, r, dst, square=True) == hg.aca_rect_s(x0, y0, w, r, dst)
    # zero offsets give a multiple of the identity
    src = hg.rect_corners(Fraction(0), Fraction(0), Fraction(127), Fraction(1))
    assert proportional(hg.aca_rect_s(0, 0, Fraction(127), Fraction(1), src, square=True),
                        [[1, 0, 0], [0, 1, 0], [0, 0, 1]])


def test_rect_all_vertex_orderings():
    # general ACA gives the same homography for all 24 orderings of a rectangle's corners
    src = hg.rect_corners(Fraction(3), Fraction(5), Fraction(40), Fraction(4, 3))
    dst = [Fraction(v) for v in (10, 12, 61, 8, 14, 47, 55, 52)]
    ref = hg.dlt_s(src, dst)
    for perm in itertools.permutations(range(4)):
        s = [src[2 * p + c] for p in perm for c in (0, 1)]
        d = [dst[2 * p + c] for p in perm for c in (0, 1)]
        assert proportional(hg.aca_s(s, d), ref)


def test_affine_special_case():
    rng = np.random.default_rng(11)
    for _ in range(100):
        A = [[int(v) for v in rng.integers(-5, 6, 3)] for _ in range(2)]
        src = [Fraction(int(v)) for v in rng.integers(-20, 20, 8)]
        dst = []
        for k in range(4):
            x, y = src[2 * k], src[2 * k + 1]
            dst += [A[0][0] * x + A[0][1] * y + A[0][2], A[1][0] * x + A[1][1] * y + A[1][2]]
        if not generic(src, dst):
            continue
        H = hg.aca_s(src, dst)
        assert H[2][0] == 0 and H[2][1] == 0
        HA = hg.affine_aca_s(src[:6], dst[:6])
        assert proportional(H, HA)
        # textbook: [N2 P2 M2; 1 1 1] [N1 P1 M1; 1 1 1]^-1
        T2 = [[dst[2], dst[4], dst[0]], [dst[3], dst[5], dst[1]], [1, 1, 1]]
        T1 = [[src[2], src[4], src[0]], [src[3], src[5], src[1]], [1, 1, 1]]
        # verify HA T1 = k T2 instead of inverting
        assert proportional(hg.matmul3(HA, T1), T2)


def test_flop_counts():
    src, dst, _ = synth.quadruples(1, 0)
    s, d = [float(v) for v in src[:, 0]], [float(v) for v in dst[:, 0]]
    H, c = flops.count(hg.aca_s, s, d)
    assert c.flops == 85 and c.div == 0                      # Table IV, up to scale
    # normalisation by h33: one division and eight multiplications (12 FLOPs)
    inv = 1 / H[2][2]
    _ = [H[i][j] * inv for i in range(3) for j in range(3) if (i, j) != (2, 2)]
    assert c.flops == 97
    _, c = flops.count(lambda a, b: hg.aca_rect_s(0.0, 0.0, 127.0, 1.0, b, square=True), s, d)
    assert c.flops == 44
    _, c = flops.count(lambda a, b, xx, yy, ww, rr: hg.aca_rect_s(xx, yy, ww, rr, b), s, d, 1.0, 2.0, 100.0, 1.5)
    assert c.flops == 47
    _, c = flops.count(hg.affine_aca_s, s[:6], d[:6])
    assert c.flops == 33
    # SKS: Table III gives 157; this transcription spends 16 (not 14) on each of
    # the Q7 and Q8 steps, all other steps match the table
    _, c = flops.count(hg.sks_s, s, d)
    assert c.flops == 161 and c.div == 6
    # simplified SK per image (the pattern constants are paid once): Table III
    # gives 73; the same two extra operations in the Q8 step give 75
    pat = hg.sk_pattern_s(s)
    _, c = flops.count(lambda b: hg.sk_simplified_s(pat, b), d)
    assert c.flops == 75 and c.div == 2
    # normalised affine: 33 plus one division and six multiplications
    _, c = flops.count(hg.affine_normalised_s, s[:6], d[:6])
    assert c.flops == 43 and c.div == 1


def test_aca64_fp64_error_against_exact():
    src, dst, _ = synth.quadruples(4096, 0)
    H = hg.aca64(src.astype(np.float64), dst.astype(np.float64))
    Hs = hg.aca64(src, dst)                      # float32 emulation, context only
    rng = np.random.default_rng(0)
    sel = rng.choice(4096, 96, replace=False)
    e64, e32 = [], []
    for i in sel:
        Hx = hg.exact_h(src[:, i], dst[:, i])
        e64.append(float(hg.herr(H[i], Hx)))
        e32.append(float(hg.herr(Hs[i], Hx)))
    assert max(e64) < 1e-11
    assert max(e32) > 1e-7             # single precision is visibly worse


def test_aca64_equals_scalar_and_dlt64():
    src, dst, _ = synth.quadruples(512, 3)
    H = hg.aca64(src.astype(np.float64), dst.astype(np.float64))
    for i in range(0, 512, 64):
        Hs = hg.aca_s([float(v) for v in src[:, i]], [float(v) for v in dst[:, i]])
        assert np.array_equal(np.array(Hs), H[i])
    assert hg.herr(H, hg.dlt64(src, dst)).max() < 1e-9
    S = hg.sks64(src.astype(np.float64), dst.astype(np.float64))
    assert hg.herr(S, H).max() < 1e-9


def test_degeneracy_flag():
    # exactly collinear integer triples on either side are flagged
    src = np.array([[0, 0, 10, 0, 0, 10, 20, 0]], np.float32).T      # M N Q collinear
    dst = np.array([[1, 2, 11, 3, 2, 15, 19, 19]], np.float32).T
    assert hg.degeneracy_flags(src, dst)[0] == hg.FLAG_NEAR_DEGENERATE
    assert hg.degeneracy_flags(dst, src)[0] == hg.FLAG_NEAR_DEGENERATE
    assert hg.degeneracy_flags(dst, dst)[0] == 0
    bad = dst.copy()
    bad[3, 0] = np.nan
    assert hg.degeneracy_flags(bad, dst)[0] == hg.FLAG_NONFINITE_INPUT
    # min height by brute force: a right triangle 3-4-5 has height 12/5 over the hypotenuse
    q = np.array([[0, 0, 3, 0, 0, 4, 50, 50]], np.float64).T
    assert abs(hg.side_heights(q)[0, 0] - 2.4) < 1e-12
    # planted near-degenerate sets are all flagged
    s, d, lab = synth.quadruples(20000, 1, degenerate_every=100)
    f = hg.degeneracy_flags(s, d)
    assert lab.sum() == 200
    assert np.all(f[lab == 1] & 1)
    assert (f[lab == 0] & 1).sum() <= 10


def test_pow2_scaling():
    rng = np.random.default_rng(2)
    H = rng.normal(size=(1000, 3, 3)) * np.exp(rng.uniform(-60, 60, (1000, 1, 1)))
    H32, ok = hg.pow2_f32(H)
    assert ok.all()
    m = np.abs(H32).max(axis=(1, 2))
    assert np.all((m >= 0.5) & (m <= 1.0))
    e = np.frexp(np.abs(H).max(axis=(1, 2)))[1]
    assert np.array_equal(H32, np.ldexp(H, -e[:, None, None]).astype(np.float32))
    Z, ok = hg.pow2_f32(np.zeros((2, 3, 3)))
    assert not ok.any() and not Z.any()


def test_herr_scale_and_sign():
    rng = np.random.default_rng(3)
    H = rng.normal(size=(10, 3, 3))
    assert hg.herr(H, -3.5 * H).max() < 1e-15
    assert hg.herr(H, H + 1e-3).min() > 1e-5
