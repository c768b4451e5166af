"""Simplified SK (known pattern, many images) and the three-point affine on the
GPU against the oracle (parity tests).

Bar, as for the 4-point solvers: on every problem not flagged near-degenerate
the result agrees with the float64 oracle within 1e-5 (Hbar up to scale,
Frobenius-normalised and sign-fixed; the affine map entrywise, its linear part
relative to that part's norm and its translation relative to the size of the
terms it cancels) and with the plain definition (the normalised DLT through the four
correspondences after composing with H_S1; the 3 x 3 linear solve for the
affine map); flag bits agree except where the oracle's minimum triangle height
lies within a relative 1e-3 of the 1e-2 threshold."""
import numpy as np
import pytest
import torch

import synth
from oracle import homography as hg
from tests.gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-5
OBJ = synth.PATTERN


def near_threshold(h):
    return np.abs(h - hg.DELTA_PX) <= 1e-3 * hg.DELTA_PX


def to_gpu(planes, k, ld=None, offset=0):
    n = planes.shape[1]
    ld = n if ld is None else ld
    T = torch.full((k, ld + offset), float("nan"), device="cuda")
    T[:, offset:offset + n] = torch.from_numpy(planes)
    return T[:, offset:offset + n]


# ---- simplified SK ------------------------------------------------------------

def gpu_sk(obj, dst, ld=None, offset=0):
    import paper_2402_18008_amd as hgpu
    n = dst.shape[1]
    H, f, frame = hgpu.hg_solve_sk(obj, to_gpu(dst, 8, ld, offset))
    torch.cuda.synchronize()
    return H.cpu().numpy().T.reshape(n, 3, 3), f.cpu().numpy(), frame


def check_sk(obj, dst, Hg, fg, frame, label=""):
    Hb, HS1 = hg.sk64(obj, dst)
    assert np.array_equal(frame, HS1), label
    H32, ok = hg.pow2_f32(Hb)
    fo = hg.sk_flags(obj, dst) | np.where(ok, 0, hg.FLAG_ZERO_H).astype(np.uint8)
    pat_h = hg.side_heights(np.asarray(obj, np.float64)[:, None]).min()
    mh = np.minimum(hg.side_heights(dst).min(axis=0), pat_h)
    bad = (fg != fo) & ~near_threshold(mh)
    assert not bad.any(), (label, np.nonzero(bad)[0][:10], fg[bad][:10], fo[bad][:10])
    sel = (fo == 0) & (fg == 0)
    e = hg.herr(Hg[sel], H32[sel].astype(np.float64))
    assert e.max() <= TOL, (label, e.max())
    # the plain definition: Hbar H_S1 is the homography through the 4 correspondences
    src = np.repeat(np.asarray(obj, np.float64)[:, None], int(sel.sum()), axis=1)
    e2 = hg.herr(Hg[sel].astype(np.float64) @ HS1, hg.dlt64(src, dst[:, sel]))
    assert e2.max() <= TOL, (label, e2.max())
    return dict(max_err=float(e.max()), exact=float((Hg[sel] == H32[sel]).all(axis=(1, 2)).mean()))


def test_sk_pattern_images():
    require_gpu()
    dst = synth.pattern_images(4096, 10)
    announce("solve_sk pattern images n=4096")
    Hg, fg, frame = gpu_sk(OBJ, dst)
    st = check_sk(OBJ, dst, Hg, fg, frame, "sk4096")
    print("sk", st)
    assert st["exact"] > 0.99          # same operation order in double precision


@pytest.mark.parametrize("n,ld,offset", [(1, 1, 0), (3, 3, 0), (5, 8, 0), (4097, 4100, 0),
                                         (1029, 1029, 1), (777, 800, 3)])
def test_sk_ragged_and_unaligned(n, ld, offset):
    require_gpu()
    dst = synth.pattern_images(n, 200 + n)
    announce(f"solve_sk n={n} ld={ld} offset={offset}")
    Hg, fg, frame = gpu_sk(OBJ, dst, ld, offset)
    check_sk(OBJ, dst, Hg, fg, frame, f"n={n}")


def test_sk_other_patterns():
    """Patterns given in other object frames (a canonical one among them) and
    random image quadruples, not only images of the default pattern."""
    require_gpu()
    _, dst, _ = synth.quadruples(2048, 11)
    for obj in ([-1.0, 0.0, 1.0, 0.0, 0.3, 0.7, -0.2, 0.5],
                [500.0, -20.0, 120.0, 40.0, 300.0, 310.0, 90.0, 260.0]):
        announce(f"solve_sk pattern {obj}")
        Hg, fg, frame = gpu_sk(obj, dst)
        check_sk(obj, dst, Hg, fg, frame, str(obj))


def test_sk_degenerate():
    require_gpu()
    dst = synth.pattern_images(64, 12)
    dst[:, 0] = [0, 0, 10, 10, 20, 20, 5, 40]          # image M N P collinear
    dst[:, 1] = [1, 1, 1, 1, 50, 60, 70, 10]           # image M == N
    dst[3, 2] = np.nan
    announce("solve_sk degenerate images")
    Hg, fg, frame = gpu_sk(OBJ, dst)
    assert fg[0] & 1 and fg[1] & 1
    assert fg[2] == 6 and not Hg[2].any()
    check_sk(OBJ, dst[:, 3:], Hg[3:], fg[3:], frame)
    # a pattern with three collinear points: every image flagged, Hbar zero (bit2)
    obj = [0.0, 0.0, 100.0, 0.0, 50.0, 0.0, 120.0, 90.0]
    announce("solve_sk collinear pattern")
    Hg, fg, _ = gpu_sk(obj, dst[:, 3:])
    assert np.all(fg & 1) and np.all(fg & 4) and not Hg.any()


def test_sk_empty_writes_frame():
    require_gpu()
    import paper_2402_18008_amd as hgpu
    H, f, frame = hgpu.hg_solve_sk(OBJ, torch.empty((8, 0), device="cuda"))
    assert H.shape == (9, 0) and f.shape == (0,)
    assert np.array_equal(frame, hg.sk64(OBJ, np.zeros((8, 0)))[1])


def test_sk_full_size_sampled():
    """2^26 images in the launch the benchmark times; a 1-in-1024 sample plus
    every flagged image match the oracle."""
    require_gpu()
    import paper_2402_18008_amd as hgpu
    n = 1 << 26
    announce("solve_sk generating 2^26 pattern images")
    dst = synth.pattern_images(n, 1, workers=16)
    D = torch.from_numpy(dst).cuda()
    announce("solve_sk 2^26 launch")
    H, f, frame = hgpu.hg_solve_sk(OBJ, D)
    torch.cuda.synchronize()
    fg = f.cpu().numpy()
    sel = np.unique(np.concatenate([np.arange(0, n, 1024), np.nonzero(fg)[0][:20000]]))
    Hs = H[:, torch.from_numpy(sel).cuda()].cpu().numpy().T.reshape(-1, 3, 3)
    st = check_sk(OBJ, dst[:, sel], Hs, fg[sel], frame, "sk 2^26")
    print("sk 2^26", st, "flagged", int((fg != 0).sum()))
    del D, H, f


# ---- three-point affine ---------------------------------------------------------

def gpu_affine(src, dst, ld=None, offset=0):
    import paper_2402_18008_amd as hgpu
    n = src.shape[1]
    A, f = hgpu.hg_solve3_affine(to_gpu(src, 6, ld, offset), to_gpu(dst, 6, ld, offset))
    torch.cuda.synchronize()
    return A.cpu().numpy().T.reshape(n, 2, 3), f.cpu().numpy()


def textbook_affine(src, dst):
    """[A | t] from the 3 x 3 linear system [x y 1] (a_i1, a_i2, a_i3) = x'_i."""
    n = src.shape[1]
    S = np.stack([src[0::2].T, src[1::2].T, np.ones((n, 3))], axis=2)     # (n, 3, 3)
    rhs = np.stack([dst[0::2].T, dst[1::2].T], axis=2)                    # (n, 3, 2)
    return np.linalg.solve(S, rhs).transpose(0, 2, 1)                      # (n, 2, 3)


def aff_err(A, B, src):
    """Entrywise error of A against B (n, 2, 3): the linear part relative to
    the Frobenius norm of B's linear part, the translation relative to
    |t| + ||B_lin|| R, with R the largest source coordinate magnitude (the size
    of the terms a translation cancels)."""
    lin = np.linalg.norm(B[:, :, :2].reshape(len(B), -1), axis=1)
    R = np.maximum(np.abs(src).max(axis=0), 1.0)
    e_lin = np.abs(A[:, :, :2] - B[:, :, :2]).max(axis=(1, 2)) / lin
    e_t = (np.abs(A[:, :, 2] - B[:, :, 2]) / (np.abs(B[:, :, 2]) + (lin * R)[:, None])).max(axis=1)
    return np.maximum(e_lin, e_t)


def check_affine(src, dst, Ag, fg, label=""):
    s64, d64 = src.astype(np.float64), dst.astype(np.float64)
    Ao = hg.affine64(s64, d64)
    fin = np.isfinite(Ao).all(axis=(1, 2))
    A32 = np.where(fin[:, None, None], Ao, 0.0).astype(np.float32)
    fo = hg.affine_flags(src, dst) | np.where(fin, 0, hg.FLAG_ZERO_H).astype(np.uint8)
    mh = np.minimum(hg.triangle_heights(s64), hg.triangle_heights(d64))
    bad = (fg != fo) & ~near_threshold(mh)
    assert not bad.any(), (label, np.nonzero(bad)[0][:10], fg[bad][:10], fo[bad][:10])
    sel = (fo == 0) & (fg == 0)
    e = aff_err(Ag[sel].astype(np.float64), A32[sel].astype(np.float64), s64[:, sel])
    assert e.max() <= TOL, (label, e.max())
    e2 = aff_err(Ag[sel].astype(np.float64), textbook_affine(s64[:, sel], d64[:, sel]), s64[:, sel])
    assert e2.max() <= TOL, (label, e2.max())
    return dict(max_err=float(e.max()), exact=float((Ag[sel] == A32[sel]).all(axis=(1, 2)).mean()))


def test_affine_config0_triangles():
    require_gpu()
    src, dst, _ = synth.config0()
    announce("solve3_affine n=4096")
    Ag, fg = gpu_affine(src[:6], dst[:6])
    st = check_affine(src[:6], dst[:6], Ag, fg, "affine4096")
    print("affine", st)
    assert st["exact"] > 0.99


@pytest.mark.parametrize("n,ld,offset", [(1, 1, 0), (3, 3, 0), (5, 8, 0), (4097, 4100, 0),
                                         (1029, 1029, 1), (777, 800, 3)])
def test_affine_ragged_and_unaligned(n, ld, offset):
    require_gpu()
    src, dst, _ = synth.quadruples(n, 300 + n)
    announce(f"solve3_affine n={n} ld={ld} offset={offset}")
    Ag, fg = gpu_affine(src[:6], dst[:6], ld, offset)
    check_affine(src[:6], dst[:6], Ag, fg, f"n={n}")


def test_affine_exact_on_integer_maps():
    """Integer affine maps of integer triangles come back exactly."""
    require_gpu()
    rng = np.random.default_rng(13)
    n = 512
    src = rng.integers(-200, 200, (6, n)).astype(np.float32)
    A = rng.integers(-4, 5, (n, 2, 3)).astype(np.float64)
    dst = np.empty_like(src)
    for k in range(3):
        x, y = src[2 * k].astype(np.float64), src[2 * k + 1].astype(np.float64)
        dst[2 * k] = A[:, 0, 0] * x + A[:, 0, 1] * y + A[:, 0, 2]
        dst[2 * k + 1] = A[:, 1, 0] * x + A[:, 1, 1] * y + A[:, 1, 2]
    announce("solve3_affine integer maps n=512")
    Ag, fg = gpu_affine(src, dst)
    ok = (fg & 4) == 0
    assert ok.mean() > 0.95
    assert np.array_equal(Ag[ok], A[ok].astype(np.float32))


def test_affine_degenerate():
    require_gpu()
    src, dst, _ = synth.quadruples(64, 14)
    src, dst = src[:6].copy(), dst[:6].copy()
    src[:, 0] = [0, 0, 10, 10, 20, 20]                 # source triangle collinear: no affine
    dst[:, 1] = [0, 0, 10, 10, 20, 20]                 # target collinear: singular but defined
    dst[4, 2] = np.inf
    announce("solve3_affine degenerate")
    Ag, fg = gpu_affine(src, dst)
    assert fg[0] == 5 and not Ag[0].any()
    assert fg[1] == 1 and np.isfinite(Ag[1]).all()
    assert fg[2] == 6 and not Ag[2].any()
    check_affine(src[:, 3:], dst[:, 3:], Ag[3:], fg[3:])


def test_affine_full_size_sampled():
    """2^26 triangles (the first three points of the 2^26-quadruple workload,
    with its planted near-degenerate sets) in the launch the benchmark times."""
    require_gpu()
    import paper_2402_18008_amd as hgpu
    n = 1 << 26
    announce("solve3_affine generating 2^26 quadruples")
    src, dst, _ = synth.config1(n, workers=16)
    S = torch.from_numpy(src[:6]).cuda()
    D = torch.from_numpy(dst[:6]).cuda()
    announce("solve3_affine 2^26 launch")
    A, f = hgpu.hg_solve3_affine(S, D)
    torch.cuda.synchronize()
    fg = f.cpu().numpy()
    sel = np.unique(np.concatenate([np.arange(0, n, 1024), np.nonzero(fg)[0][:20000]]))
    As = A[:, torch.from_numpy(sel).cuda()].cpu().numpy().T.reshape(-1, 2, 3)
    st = check_affine(src[:6, sel], dst[:6, sel], As, fg[sel], "affine 2^26")
    print("affine 2^26", st, "flagged", int((fg != 0).sum()))
    del S, D, A, f
