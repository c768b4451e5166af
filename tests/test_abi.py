"""The C ABI: the library loads, exports every declared entry point, and its
host-side argument checks reject bad input before touching the GPU (CPU only)."""
import ctypes as C
import os
import re

import pytest

from paper_2402_18008_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "homog.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2402_18008_amd import build
        build.build()
    return _abi.lib()


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hg_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(names) <= set(_abi.SIGNATURES)


def test_status_strings(lib):
    assert lib.hg_version() >= 10000
    for st in (0, -1, -2, -3, -4):
        assert lib.hg_status_str(st)


FAKE = C.c_void_p(0x1000)   # never dereferenced: validation fails first


def test_solve4_validation(lib):
    f = lib.hg_solve4
    assert f(7, FAKE, FAKE, 10, 10, FAKE, None, None) == _abi.HG_EINVAL
    assert b"method" in lib.hg_last_error()
    assert f(0, FAKE, FAKE, -1, 10, FAKE, None, None) == _abi.HG_EINVAL
    assert f(0, FAKE, FAKE, 10, 9, FAKE, None, None) == _abi.HG_EINVAL
    assert f(0, None, FAKE, 10, 10, FAKE, None, None) == _abi.HG_EINVAL
    assert f(0, FAKE, FAKE, 10, 10, None, None, None) == _abi.HG_EINVAL
    # n == 0 is a no-op even with NULL pointers
    assert f(0, None, None, 0, 0, None, None, None) == _abi.HG_OK
    assert f(1, None, None, 0, 0, None, None, None) == _abi.HG_OK


def test_sk_and_affine_validation(lib):
    D8 = C.c_double * 8
    obj = D8(0.0, 0.0, 100.0, 0.0, 0.0, 80.0, 120.0, 90.0)
    f = lib.hg_solve_sk
    assert f(None, FAKE, 10, 10, FAKE, None, None, None) == _abi.HG_EINVAL
    bad = D8(*obj)
    bad[5] = float("nan")
    assert f(bad, FAKE, 10, 10, FAKE, None, None, None) == _abi.HG_EINVAL
    assert b"pattern" in lib.hg_last_error()
    assert f(obj, FAKE, -1, 10, FAKE, None, None, None) == _abi.HG_EINVAL
    assert f(obj, FAKE, 10, 9, FAKE, None, None, None) == _abi.HG_EINVAL
    assert f(obj, None, 10, 10, FAKE, None, None, None) == _abi.HG_EINVAL
    assert f(obj, FAKE, 10, 10, None, None, None, None) == _abi.HG_EINVAL
    g = lib.hg_solve3_affine
    assert g(FAKE, FAKE, -1, 10, FAKE, None, None) == _abi.HG_EINVAL
    assert g(FAKE, FAKE, 10, 9, FAKE, None, None) == _abi.HG_EINVAL
    assert g(None, FAKE, 10, 10, FAKE, None, None) == _abi.HG_EINVAL
    assert g(FAKE, FAKE, 10, 10, None, None, None) == _abi.HG_EINVAL
    assert g(None, None, 0, 0, None, None, None) == _abi.HG_OK


def test_sk_frame_host_setup(lib):
    """n == 0 runs only the host-side pattern set-up: the returned frame is the
    similarity H_S1 of the pattern (host logic; no GPU involved)."""
    import numpy as np
    from oracle import homography as hg
    vals = (3.0, -2.0, 101.5, 7.25, 10.0, 80.0, 120.0, 95.0)
    frame = (C.c_double * 9)()
    assert lib.hg_solve_sk((C.c_double * 8)(*vals), None, 0, 0, None, None, frame, None) == 0
    ref = np.array(hg.sk_pattern_s(list(vals))[4], dtype=np.float64)
    assert np.array_equal(np.array(list(frame)).reshape(3, 3), ref)


def test_general_aca_validation(lib):
    assert lib.hg_aca_fwd(FAKE, FAKE, -1, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_aca_fwd(None, FAKE, 4, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_aca_fwd(FAKE, FAKE, 4, None, None) == _abi.HG_EINVAL
    assert lib.hg_aca_fwd(None, None, 0, None, None) == _abi.HG_OK
    assert lib.hg_aca_bwd(FAKE, FAKE, FAKE, -1, FAKE, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_aca_bwd(FAKE, FAKE, None, 4, FAKE, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_aca_bwd(FAKE, FAKE, FAKE, 4, None, None, None) == _abi.HG_EINVAL
    assert b"NULL" in lib.hg_last_error()
    assert lib.hg_aca_bwd(None, None, None, 0, None, None, None) == _abi.HG_OK
    # batch limits (one thread per problem, 64-bit offsets): at most 2^30 problems
    assert lib.hg_aca_fwd(FAKE, FAKE, (1 << 30) + 1, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_aca_bwd(FAKE, FAKE, FAKE, (1 << 30) + 1, FAKE, FAKE, None) == _abi.HG_EINVAL
    assert b"2^30" in lib.hg_last_error()


def test_refine_and_photometric_validation(lib):
    f = lib.hg_refine

    def call(**kw):
        a = dict(img=FAKE, tgt=FAKE, B=16, h=32, w=32, it=6, step=1.0, off=FAKE, loss=None)
        a.update(kw)
        return f(a["img"], a["tgt"], a["B"], a["h"], a["w"], a["it"], a["step"], a["off"],
                 a["loss"], None)

    assert call(B=-1) == _abi.HG_EINVAL
    assert call(h=1) == _abi.HG_EINVAL
    assert call(it=-1) == _abi.HG_EINVAL
    assert call(it=1001) == _abi.HG_EINVAL
    assert call(step=float("nan")) == _abi.HG_EINVAL
    assert call(off=None) == _abi.HG_EINVAL
    assert call(B=0, img=None, tgt=None, off=None) == _abi.HG_OK
    out = C.c_void_p()
    assert lib.hg_refine_graph_create(FAKE, FAKE, 0, 32, 32, 6, 1.0, FAKE, None, None,
                                      C.byref(out)) == _abi.HG_EINVAL
    assert not out.value
    pf, pb = lib.hg_photometric_fwd, lib.hg_photometric_bwd
    assert pf(FAKE, FAKE, FAKE, -1, 32, 32, FAKE, None) == _abi.HG_EINVAL
    assert pf(FAKE, FAKE, FAKE, 4, 1, 32, FAKE, None) == _abi.HG_EINVAL
    assert pf(None, FAKE, FAKE, 4, 32, 32, FAKE, None) == _abi.HG_EINVAL
    assert pf(FAKE, FAKE, FAKE, 4, 32, 32, None, None) == _abi.HG_EINVAL
    assert pb(FAKE, FAKE, FAKE, None, 4, 32, 32, FAKE, None) == _abi.HG_EINVAL
    assert pb(FAKE, FAKE, FAKE, FAKE, 4, 32, 32, None, None) == _abi.HG_EINVAL
    assert pf(None, None, None, 0, 32, 32, None, None) == _abi.HG_OK
    # at most 2^27 patches per call (per-patch offsets stay 32-bit)
    big = (1 << 27) + 1
    assert pf(FAKE, FAKE, FAKE, big, 2, 2, FAKE, None) == _abi.HG_EINVAL
    assert b"2^27" in lib.hg_last_error()
    assert pb(FAKE, FAKE, FAKE, FAKE, big, 2, 2, FAKE, None) == _abi.HG_EINVAL
    assert call(B=big, h=2, w=2) == _abi.HG_EINVAL
    assert lib.hg_aca_rect_fwd(FAKE, big, 0.0, 0.0, 128.0, 1.0, FAKE, None) == _abi.HG_EINVAL


def test_ransac_validation(lib):
    f = lib.hg_ransac
    ws_need = lib.hg_ransac_ws_bytes(2000, 4096)
    assert ws_need > 0
    args = dict(corr=FAKE, n=2000, ld=2000, nh=4096, th=3.0, seed=1, bh=FAKE, bc=FAKE, bi=FAKE,
                mask=FAKE, hc=None, ws=C.c_void_p(0x100000), wsb=ws_need)

    def call(fn=f, **kw):
        a = dict(args, **kw)
        return fn(a["corr"], a["n"], a["ld"], a["nh"], a["th"], a["seed"], a["bh"], a["bc"], a["bi"],
                  a["mask"], a["hc"], a["ws"], a["wsb"], None)

    for fn in (lib.hg_ransac, lib.hg_ransac_plain):
        assert call(fn, n=3) == _abi.HG_EINVAL
        assert call(fn, ld=1999) == _abi.HG_EINVAL
        assert call(fn, nh=0) == _abi.HG_EINVAL
        assert call(fn, th=0.0) == _abi.HG_EINVAL
        assert call(fn, th=float("nan")) == _abi.HG_EINVAL
        assert call(fn, th=float("inf")) == _abi.HG_EINVAL
        assert call(fn, th=1e-39) == _abi.HG_EINVAL
        assert call(fn, corr=None) == _abi.HG_EINVAL
        assert call(fn, mask=None) == _abi.HG_EINVAL
        assert call(fn, ws=None) == _abi.HG_EWORKSPACE
        assert call(fn, wsb=ws_need - 1) == _abi.HG_EWORKSPACE
        assert call(fn, ws=C.c_void_p(0x100008)) == _abi.HG_EINVAL     # misaligned


def test_batched_validation(lib):
    need = lib.hg_ransac_batched_ws_bytes(512, 1024)
    ws = C.c_void_p(0x100000)

    def call(tune=None, **kw):
        a = dict(corr=FAKE, ld=10, off=FAKE, n_pairs=512, n_hyp=1024, th=3.0, bh=FAKE, ws=ws, wsb=need)
        a.update(kw)
        return lib.hg_ransac_batched(a["corr"], a["ld"], a["off"], a["n_pairs"], a["n_hyp"], a["th"], 3,
                                     tune, a["bh"], FAKE, FAKE, FAKE, None, a["ws"], a["wsb"], None)

    assert call(n_pairs=0) == _abi.HG_EINVAL
    assert call(off=None) == _abi.HG_EINVAL
    assert call(n_hyp=0) == _abi.HG_EINVAL
    assert call(th=-1.0) == _abi.HG_EINVAL
    assert call(bh=None) == _abi.HG_EINVAL
    assert call(wsb=need - 1) == _abi.HG_EWORKSPACE
    # more than 2^31 work items would wrap the persistent queue's 32-bit counter
    assert call(n_hyp=2**31 - 1) == _abi.HG_EINVAL
    assert b"too large" in lib.hg_last_error()
    bad = _abi.Tuning(5, 16, 1, 0)
    assert call(tune=C.byref(bad)) == _abi.HG_EINVAL
    bad = _abi.Tuning(8, 48, 1, 0)
    assert call(tune=C.byref(bad)) == _abi.HG_EINVAL
    bad = _abi.Tuning(8, 16, 9, 0)
    assert call(tune=C.byref(bad)) == _abi.HG_EINVAL
    h = C.c_void_p()
    assert lib.hg_ransac_batched_graph_create(FAKE, 10, FAKE, 0, 1024, 3.0, 3, None, FAKE, FAKE, FAKE,
                                              FAKE, None, ws, need, None, C.byref(h)) == _abi.HG_EINVAL
    assert not h.value
    assert lib.hg_graph_launch(None, None) == _abi.HG_EINVAL
    lib.hg_graph_destroy(None)


def test_diff_validation(lib):
    assert lib.hg_aca_rect_fwd(FAKE, -1, 0.0, 0.0, 127.0, 1.0, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_aca_rect_fwd(FAKE, 4, 0.0, 0.0, 0.0, 1.0, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_aca_rect_fwd(FAKE, 4, 0.0, 0.0, 127.0, -1.0, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_aca_rect_fwd(None, 4, 0.0, 0.0, 127.0, 1.0, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_aca_rect_fwd(None, 0, 0.0, 0.0, 127.0, 1.0, None, None) == _abi.HG_OK
    assert lib.hg_aca_rect_bwd(FAKE, None, 4, 0.0, 0.0, 127.0, 1.0, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_warp_l1_fwd(FAKE, FAKE, FAKE, 4, 0, 128, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_warp_l1_fwd(FAKE, None, FAKE, 4, 128, 128, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_warp_l1_fwd(None, FAKE, FAKE, 4, 128, 128, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_warp_l1_fwd(None, None, None, 0, 128, 128, None, None) == _abi.HG_OK
    # at most 2^29 pixels per patch (32-bit byte offsets into the patch)
    assert lib.hg_warp_l1_fwd(None, None, None, 0, 32768, 32768, None, None) == _abi.HG_EINVAL
    assert lib.hg_warp_l1_fwd(None, None, None, 0, 16384, 32768, None, None) == _abi.HG_OK
    assert lib.hg_photometric_fwd(None, None, None, 0, 32768, 32768, None, None) == _abi.HG_EINVAL
    assert lib.hg_warp_l1_bwd(FAKE, FAKE, FAKE, None, 4, 128, 128, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_warp_store_fwd(FAKE, FAKE, 4, 128, 40000, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_l1_fwd(FAKE, FAKE, 4, 128, 128, None, None) == _abi.HG_EINVAL
    assert lib.hg_l1_bwd(FAKE, FAKE, None, 4, 128, 128, FAKE, None) == _abi.HG_EINVAL
    assert lib.hg_warp_bwd_from_grad(FAKE, FAKE, FAKE, 4, 128, 128, None, None) == _abi.HG_EINVAL


def test_stream_copy_validation(lib):
    assert lib.hg_stream_copy(FAKE, FAKE, -1, None) == _abi.HG_EINVAL
    assert lib.hg_stream_copy(None, FAKE, 5, None) == _abi.HG_EINVAL
    assert lib.hg_stream_copy(None, None, 0, None) == _abi.HG_OK


def test_stream_planes_validation(lib):
    assert lib.hg_stream_planes(FAKE, 16, FAKE, 9, None, -1, 10, None) == _abi.HG_EINVAL
    assert lib.hg_stream_planes(None, 16, None, 9, None, 0, 0, None) == _abi.HG_OK
    assert lib.hg_stream_planes(None, 16, FAKE, 9, None, 5, 5, None) == _abi.HG_EINVAL
    assert lib.hg_stream_planes(FAKE, 16, FAKE, 9, None, 5, 4, None) == _abi.HG_EINVAL
    for n_in, n_out in ((1, 1), (16, 8), (9, 9), (0, 9)):
        assert lib.hg_stream_planes(FAKE, n_in, FAKE, n_out, None, 5, 5, None) == _abi.HG_EINVAL
        assert b"unsupported shape" in lib.hg_last_error()


def test_adaptive_validation(lib):
    need = lib.hg_ransac_adaptive_ws_bytes(512, 1000)
    assert need > lib.hg_ransac_batched_ws_bytes(512, 1000)
    ws = C.c_void_p(0x100000)

    def call(**kw):
        a = dict(conf=0.99, ne=FAKE, n_pairs=512, wsb=need, th=3.0)
        a.update(kw)
        return lib.hg_ransac_adaptive(FAKE, 10, FAKE, a["n_pairs"], 1000, a["th"], 1, a["conf"], None,
                                      FAKE, FAKE, FAKE, FAKE, a["ne"], ws, a["wsb"], None)

    assert call(conf=1.0) == _abi.HG_EINVAL
    assert call(conf=0.0) == _abi.HG_EINVAL
    assert call(ne=None) == _abi.HG_EINVAL
    assert call(n_pairs=0) == _abi.HG_EINVAL
    assert call(th=0.0) == _abi.HG_EINVAL
    assert call(wsb=need - 1) == _abi.HG_EWORKSPACE
    assert lib.hg_ransac_adaptive(FAKE, 10, FAKE, 2**20, 2**20, 3.0, 1, 0.99, None, FAKE, FAKE, FAKE,
                                  FAKE, FAKE, ws, need, None) == _abi.HG_EINVAL
