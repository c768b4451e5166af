"""MI355X-native minimal 4-point homography (ACA / SKS) with fused RANSAC
scoring and a differentiable 4-point-offset pipeline.

Thin torch binding over libhomog (include/homog.h): every function marshals
device tensors into the C ABI on the current HIP stream; all computation runs
in the library's HIP kernels. Function names match the C entry points.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _abi
from ._abi import HG_ACA, HG_SKS, HomogError, Tuning  # noqa: F401

__all__ = ["hg_solve4", "solve4", "HomogError", "HG_ACA", "HG_SKS"]


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dev(t, name, dtype=torch.float32):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return t


def _planes(t, name, k):
    """(k, n) tensor of planes with unit inner stride; returns its plane stride."""
    _dev(t, name)
    if t.dim() != 2 or t.shape[0] != k or (t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError(f"{name} must be a ({k}, n) tensor with contiguous rows")
    return t.stride(0) if t.shape[0] > 1 else t.shape[1]


def hg_solve4(src, dst, method=HG_ACA, H=None, flags=None, stream=None):
    """Solve every quadruple of ``src``/``dst`` ((8, n) float32 planes xM yM xN
    yN xP yP xQ yQ sharing one plane stride). Returns (H (9, n) float32 planes
    h11..h33, flags (n,) uint8). ``method`` is HG_ACA or HG_SKS (or "aca",
    "sks")."""
    if isinstance(method, str):
        method = {"aca": HG_ACA, "sks": HG_SKS}[method.lower()]
    ld = _planes(src, "src", 8)
    if _planes(dst, "dst", 8) != ld:
        raise ValueError("src and dst must share the plane stride")
    n = src.shape[1]
    if H is None:
        H = torch.empty((9, ld), dtype=torch.float32, device=src.device)[:, :n]
    elif _planes(H, "H", 9) != ld:
        raise ValueError("H must share the plane stride of src")
    if flags is None:
        flags = torch.empty(n, dtype=torch.uint8, device=src.device)
    _dev(flags, "flags", torch.uint8)
    _abi.call("hg_solve4", int(method), src.data_ptr(), dst.data_ptr(), n, ld, H.data_ptr(),
              flags.data_ptr(), _stream(stream))
    return H, flags


solve4 = hg_solve4


def hg_solve_sk(obj, dst, H=None, flags=None, stream=None):
    """Simplified SK for one known pattern ``obj`` (8 numbers xM yM xN yN xP yP
    xQ yQ in object coordinates) and its images ``dst`` ((8, n) float32
    planes). Returns (Hbar (9, n) planes, flags (n,), H_S1 (3, 3) float64
    numpy array) with the object-to-image homography Hbar H_S1 up to scale."""
    import numpy as np
    o = (C.c_double * 8)(*[float(v) for v in obj])
    frame = (C.c_double * 9)()
    ld = _planes(dst, "dst", 8)
    n = dst.shape[1]
    if H is None:
        H = torch.empty((9, ld), dtype=torch.float32, device=dst.device)[:, :n]
    elif _planes(H, "H", 9) != ld:
        raise ValueError("H must share the plane stride of dst")
    if flags is None:
        flags = torch.empty(n, dtype=torch.uint8, device=dst.device)
    _dev(flags, "flags", torch.uint8)
    _abi.call("hg_solve_sk", o, dst.data_ptr(), n, ld, H.data_ptr(), flags.data_ptr(), frame,
              _stream(stream))
    return H, flags, np.array(list(frame), dtype=np.float64).reshape(3, 3)


def hg_solve3_affine(src, dst, A=None, flags=None, stream=None):
    """Affine map through three correspondences for every column of
    ``src``/``dst`` ((6, n) float32 planes xM yM xN yN xP yP sharing one plane
    stride). Returns (A (6, n) planes a11 a12 a13 a21 a22 a23, flags (n,))."""
    ld = _planes(src, "src", 6)
    if _planes(dst, "dst", 6) != ld:
        raise ValueError("src and dst must share the plane stride")
    n = src.shape[1]
    if A is None:
        A = torch.empty((6, ld), dtype=torch.float32, device=src.device)[:, :n]
    elif _planes(A, "A", 6) != ld:
        raise ValueError("A must share the plane stride of src")
    if flags is None:
        flags = torch.empty(n, dtype=torch.uint8, device=src.device)
    _dev(flags, "flags", torch.uint8)
    _abi.call("hg_solve3_affine", src.data_ptr(), dst.data_ptr(), n, ld, A.data_ptr(),
              flags.data_ptr(), _stream(stream))
    return A, flags


def hg_stream_copy(src, dst=None, stream=None):
    """Plain copy of a float32 tensor (reference for byte counters and the
    plain-copy streaming rate; not part of the method)."""
    _dev(src, "src")
    if not src.is_contiguous():
        raise ValueError("src must be contiguous")
    if dst is None:
        dst = torch.empty_like(src)
    _abi.call("hg_stream_copy", src.data_ptr(), dst.data_ptr(), src.numel(), _stream(stream))
    return dst


def hg_stream_planes(inp, n_out, out=None, flags=None, stream=None):
    """Move a solver's bytes without its arithmetic: (n_in, n) float32 planes
    in, (n_out, n) planes and n flag bytes out, with the solver kernels'
    launch shape (the streaming ceiling of that read/write mix; not part of the
    method). Shapes 16 -> 9, 8 -> 9 and 12 -> 6."""
    _dev(inp, "inp")
    if inp.dim() != 2 or inp.stride(1) != 1:
        raise ValueError("inp must be (n_in, n) with unit stride along n")
    n_in, n = inp.shape
    ld = inp.stride(0)
    if out is None:
        out = torch.empty((n_out, ld), dtype=torch.float32, device=inp.device)[:, :n]
    if out.shape != (n_out, n) or out.stride() != (ld, 1):
        raise ValueError("out must be (n_out, n) with the plane stride of inp")
    _dev(out, "out")
    if flags is not None:
        _dev(flags, "flags", torch.uint8)
        if flags.numel() < n or not flags.is_contiguous():
            raise ValueError("flags must be contiguous with n elements")
    _abi.call("hg_stream_planes", inp.data_ptr(), n_in, out.data_ptr(), n_out,
              None if flags is None else flags.data_ptr(), n, ld, _stream(stream))
    return out


# ---- RANSAC ----------------------------------------------------------------

def _corr_planes(corr):
    ld = _planes(corr, "corr", 4)
    return ld, corr.shape[1]


def hg_ransac_ws_bytes(n_pts, n_hyp):
    return int(_abi.lib().hg_ransac_ws_bytes(int(n_pts), int(n_hyp)))


def _ws(nbytes, device, ws):
    if ws is None:
        # 256-byte aligned: torch's caching allocator returns aligned blocks
        ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    _dev(ws, "ws", torch.uint8)
    if ws.numel() < nbytes:
        raise ValueError(f"workspace of {nbytes} bytes needed, {ws.numel()} given")
    return ws


def _ransac(name, corr, n_hyp, thresh, seed, want_counts, ws, stream):
    ld, n = _corr_planes(corr)
    dev = corr.device
    ws = _ws(hg_ransac_ws_bytes(n, n_hyp), dev, ws)
    out = dict(best_H=torch.empty(9, dtype=torch.float32, device=dev),
               best_count=torch.empty(1, dtype=torch.int32, device=dev),
               best_hyp=torch.empty(1, dtype=torch.int32, device=dev),
               mask=torch.empty(n, dtype=torch.uint8, device=dev),
               hyp_counts=(torch.empty(n_hyp, dtype=torch.int32, device=dev)
                           if want_counts else None))
    hc = out["hyp_counts"]
    _abi.call(name, corr.data_ptr(), n, ld, int(n_hyp), float(thresh), int(seed) & (2**64 - 1),
              out["best_H"].data_ptr(), out["best_count"].data_ptr(), out["best_hyp"].data_ptr(),
              out["mask"].data_ptr(), hc.data_ptr() if hc is not None else None, ws.data_ptr(),
              ws.numel(), _stream(stream))
    return out


def hg_ransac(corr, n_hyp, thresh, seed, hyp_counts=True, ws=None, stream=None):
    """Fused single-pair RANSAC. ``corr``: (4, n) float32 planes x1 y1 x2 y2.
    Returns a dict of device tensors: best_H (9,), best_count (1,), best_hyp
    (1,), mask (n,) uint8 and hyp_counts (n_hyp,) or None."""
    return _ransac("hg_ransac", corr, n_hyp, thresh, seed, hyp_counts, ws, stream)


def hg_ransac_plain(corr, n_hyp, thresh, seed, hyp_counts=True, ws=None, stream=None):
    """Unfused single-pair RANSAC (solve, score, argmax, mask kernels); same
    results as ``hg_ransac``."""
    return _ransac("hg_ransac_plain", corr, n_hyp, thresh, seed, hyp_counts, ws, stream)


def hg_ransac_noalloc(corr, n_hyp, thresh, seed, hyp_counts=True, out=None, stream=None):
    """``hg_ransac`` on the library's own static workspace (no allocation in
    the call; n_hyp <= 16384). ``out``: the result dict of a previous call to
    reuse (its tensors are overwritten), else new output tensors are made
    here. Calls that overlap on one GPU race (one workspace per GPU)."""
    ld, n = _corr_planes(corr)
    dev = corr.device
    if out is None:
        out = dict(best_H=torch.empty(9, dtype=torch.float32, device=dev),
                   best_count=torch.empty(1, dtype=torch.int32, device=dev),
                   best_hyp=torch.empty(1, dtype=torch.int32, device=dev),
                   mask=torch.empty(n, dtype=torch.uint8, device=dev),
                   hyp_counts=(torch.empty(n_hyp, dtype=torch.int32, device=dev)
                               if hyp_counts else None))
    hc = out["hyp_counts"]
    _abi.call("hg_ransac_noalloc", corr.data_ptr(), n, ld, int(n_hyp), float(thresh),
              int(seed) & (2**64 - 1), out["best_H"].data_ptr(), out["best_count"].data_ptr(),
              out["best_hyp"].data_ptr(), out["mask"].data_ptr(),
              hc.data_ptr() if hc is not None else None, _stream(stream))
    return out


def hg_ransac_batched_ws_bytes(n_pairs, n_hyp):
    return int(_abi.lib().hg_ransac_batched_ws_bytes(int(n_pairs), int(n_hyp)))


def _check_off(off, total, min_pts, name="off", off_host=None):
    """Host-side check of pair offsets: contiguous int64, non-decreasing,
    off[0] >= 0, off[-1] <= total, and every pair with at least ``min_pts``
    points. Checks ``off_host`` (the caller's host copy of off) if given,
    else copies off to the host (which waits for the stream)."""
    _c(off, name, torch.int64)
    if off.dim() != 1 or off.numel() < 1:
        raise ValueError(f"{name} must be a 1-D tensor of n_pairs + 1 offsets")
    if off_host is None:
        o = off.cpu()
    else:
        o = torch.as_tensor(off_host, dtype=torch.int64).reshape(-1)
        if o.numel() != off.numel():
            raise ValueError(f"{name}_host must have the {off.numel()} entries of {name}")
    if int(o[0]) < 0 or int(o[-1]) > total:
        raise ValueError(f"{name} must lie in [0, {total}]")
    if off.numel() > 1:
        d = o[1:] - o[:-1]
        if bool((d < min_pts).any()):
            raise ValueError(f"{name} must be non-decreasing with pairs of >= {min_pts} points")


def _out(t, name, dtype, numel, device):
    if t is None:
        return None
    _c(t, name, dtype)
    if t.numel() < numel or t.device != device:
        raise ValueError(f"{name} must hold {numel} elements on {device}")
    return t


def _tuning(tune):
    if tune is None:
        return None
    if isinstance(tune, Tuning):
        return tune
    return Tuning(*(int(v) for v in tune), *([0] * (4 - len(tune))))


def hg_refit_ho(corr, off, mask=None, H=None, n_used=None, flags=None, stream=None,
                off_host=None):
    """HO-SVD least-squares homography per pair over the masked points.
    corr (4, total) float32 planes x1 y1 x2 y2, off (n_pairs + 1,) int64 on
    the device, mask (total,) uint8 or None (all points); off_host: a host
    copy of off for the checks (else off is copied back, which waits for the
    stream). Returns (H (n_pairs, 9) float32, n_used (n_pairs,) int32, flags
    (n_pairs,) uint8)."""
    ld, total = _corr_planes(corr)
    _check_off(off, total, 0, off_host=off_host)
    n_pairs = off.numel() - 1
    dev = corr.device
    if mask is not None:
        _c(mask, "mask", torch.uint8)
        if mask.numel() < total:
            raise ValueError("mask must cover every point")
    H = _out(H, "H", torch.float32, 9 * n_pairs, dev)
    n_used = _out(n_used, "n_used", torch.int32, n_pairs, dev)
    flags = _out(flags, "flags", torch.uint8, n_pairs, dev)
    H = torch.empty((n_pairs, 9), dtype=torch.float32, device=dev) if H is None else H
    n_used = torch.empty(n_pairs, dtype=torch.int32, device=dev) if n_used is None else n_used
    flags = torch.empty(n_pairs, dtype=torch.uint8, device=dev) if flags is None else flags
    _abi.call("hg_refit_ho", corr.data_ptr(), ld, off.data_ptr(), n_pairs,
              mask.data_ptr() if mask is not None else None, H.data_ptr(), n_used.data_ptr(),
              flags.data_ptr(), _stream(stream))
    return H, n_used, flags


class BatchedRansac:
    """Device buffers and launcher for RANSAC over many uneven pairs.

    ``corr`` (4, total) float32 planes; ``off`` (n_pairs + 1,) int64 on the
    device. Outputs (allocated here): best_H (n_pairs, 9), best_count,
    best_hyp (n_pairs,), mask (total,) and hyp_counts (n_pairs, n_hyp) or None.
    """

    def __init__(self, corr, off, n_hyp, thresh, seed, hyp_counts=False):
        self.ld, self.total = _corr_planes(corr)
        _check_off(off, self.total, 4)
        self.corr, self.off = corr, off
        self.n_pairs = off.numel() - 1
        self.n_hyp, self.thresh, self.seed = int(n_hyp), float(thresh), int(seed) & (2**64 - 1)
        dev = corr.device
        self.ws = _ws(hg_ransac_batched_ws_bytes(self.n_pairs, self.n_hyp), dev, None)
        self.best_H = torch.empty((self.n_pairs, 9), dtype=torch.float32, device=dev)
        self.best_count = torch.empty(self.n_pairs, dtype=torch.int32, device=dev)
        self.best_hyp = torch.empty(self.n_pairs, dtype=torch.int32, device=dev)
        self.mask = torch.empty(self.total, dtype=torch.uint8, device=dev)
        self.hyp_counts = (torch.empty((self.n_pairs, self.n_hyp), dtype=torch.int32, device=dev)
                           if hyp_counts else None)

    def _args(self):
        hc = self.hyp_counts
        return (self.best_H.data_ptr(), self.best_count.data_ptr(), self.best_hyp.data_ptr(),
                self.mask.data_ptr(), hc.data_ptr() if hc is not None else None,
                self.ws.data_ptr(), self.ws.numel())

    def run(self, tune=None, stream=None):
        """hg_ransac_batched (persistent kernel) on the current stream."""
        t = _tuning(tune)
        _abi.call("hg_ransac_batched", self.corr.data_ptr(), self.ld, self.off.data_ptr(),
                  self.n_pairs, self.n_hyp, self.thresh, self.seed,
                  None if t is None else C.byref(t), *self._args(), _stream(stream))
        return self

    def autotune(self, off_host, stream=None):
        """hg_ransac_autotune on this problem; returns (pts_per_lane,
        hyps_per_block, blocks_per_cu)."""
        oh = torch.as_tensor(off_host, dtype=torch.int64).contiguous()
        t = Tuning()
        _abi.call("hg_ransac_autotune", self.corr.data_ptr(), self.ld, self.off.data_ptr(),
                  C.c_void_p(oh.data_ptr()), self.n_pairs, self.n_hyp, self.thresh, self.seed,
                  self.ws.data_ptr(), self.ws.numel(), _stream(stream), C.byref(t))
        return (t.pts_per_lane, t.hyps_per_block, t.blocks_per_cu)

    def graph(self, tune=None, stream=None):
        """Capture into a HIP graph (hg_ransac_batched_graph_create)."""
        return RansacGraph(self, tune, stream)


class AdaptiveRansac:
    """RANSAC over many uneven pairs with adaptive termination
    (hg_ransac_adaptive): ``corr`` (4, total) float32, ``off`` (n_pairs + 1,)
    int64 on the device; outputs best_H (n_pairs, 9), best_count, best_hyp,
    n_evaluated (n_pairs,) and mask (total,)."""

    def __init__(self, corr, off, n_hyp_max, thresh, seed, confidence=0.99):
        self.ld, self.total = _corr_planes(corr)
        _check_off(off, self.total, 4)
        self.corr, self.off = corr, off
        self.n_pairs = off.numel() - 1
        self.n_hyp, self.thresh = int(n_hyp_max), float(thresh)
        self.seed, self.confidence = int(seed) & (2**64 - 1), float(confidence)
        dev = corr.device
        nb = int(_abi.lib().hg_ransac_adaptive_ws_bytes(self.n_pairs, self.n_hyp))
        self.ws = _ws(nb, dev, None)
        self.best_H = torch.empty((self.n_pairs, 9), dtype=torch.float32, device=dev)
        self.best_count = torch.empty(self.n_pairs, dtype=torch.int32, device=dev)
        self.best_hyp = torch.empty(self.n_pairs, dtype=torch.int32, device=dev)
        self.n_evaluated = torch.empty(self.n_pairs, dtype=torch.int32, device=dev)
        self.mask = torch.empty(self.total, dtype=torch.uint8, device=dev)

    def run(self, tune=None, stream=None):
        t = _tuning(tune)
        _abi.call("hg_ransac_adaptive", self.corr.data_ptr(), self.ld, self.off.data_ptr(),
                  self.n_pairs, self.n_hyp, self.thresh, self.seed, self.confidence,
                  None if t is None else C.byref(t), self.best_H.data_ptr(),
                  self.best_count.data_ptr(), self.best_hyp.data_ptr(), self.mask.data_ptr(),
                  self.n_evaluated.data_ptr(), self.ws.data_ptr(), self.ws.numel(),
                  _stream(stream))
        return self


class Graph:
    """A captured launch sequence (hg_graph); ``owner`` keeps the captured
    buffers alive for as long as the graph exists."""

    def __init__(self, handle, owner):
        self.h = handle
        self.owner = owner

    def launch(self, stream=None):
        _abi.call("hg_graph_launch", self.h, _stream(stream))

    def close(self):
        if self.h:
            _abi.lib().hg_graph_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RansacGraph(Graph):
    """hg_ransac_batched captured for replay (the BatchedRansac's buffers)."""

    def __init__(self, br, tune=None, stream=None):
        t = _tuning(tune)
        h = C.c_void_p()
        _abi.call("hg_ransac_batched_graph_create", br.corr.data_ptr(), br.ld, br.off.data_ptr(),
                  br.n_pairs, br.n_hyp, br.thresh, br.seed, None if t is None else C.byref(t),
                  *br._args(), _stream(stream), C.byref(h))
        super().__init__(h, br)


# ---- differentiable 4-point-offset pipeline ----------------------------------

def _c(t, name, dtype=torch.float32):
    _dev(t, name, dtype)
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def hg_aca_rect_fwd(offsets, x0, y0, w, r, stream=None):
    """H (B, 9) float64 from offsets (B, 4, 2) float32 [TL, TR, BR, BL] by
    ACA with the source corners at the rectangle's."""
    _c(offsets, "offsets")
    B = offsets.shape[0]
    H = torch.empty((B, 9), dtype=torch.float64, device=offsets.device)
    _abi.call("hg_aca_rect_fwd", offsets.data_ptr(), B, float(x0), float(y0), float(w), float(r),
              H.data_ptr(), _stream(stream))
    return H


def hg_aca_rect_bwd(offsets, grad_H, x0, y0, w, r, stream=None):
    _c(offsets, "offsets")
    _c(grad_H, "grad_H", torch.float64)
    B = offsets.shape[0]
    g = torch.empty((B, 4, 2), dtype=torch.float32, device=offsets.device)
    _abi.call("hg_aca_rect_bwd", offsets.data_ptr(), grad_H.data_ptr(), B, float(x0), float(y0),
              float(w), float(r), g.data_ptr(), _stream(stream))
    return g


def _quad_rows(t, name):
    _c(t, name)
    if t.dim() < 2 or t.shape[-1] * (t.shape[-2] if t.dim() == 3 else 1) != 8:
        raise ValueError(f"{name} must be (B, 8) or (B, 4, 2)")
    return t.shape[0]


def hg_aca_fwd(src, dst, stream=None):
    """H (B, 9) float64 at ACA's own scale from general quadrilaterals src,
    dst ((B, 8) or (B, 4, 2) float32, points M N P Q)."""
    B = _quad_rows(src, "src")
    if _quad_rows(dst, "dst") != B:
        raise ValueError("src and dst must have the same batch size")
    H = torch.empty((B, 9), dtype=torch.float64, device=src.device)
    _abi.call("hg_aca_fwd", src.data_ptr(), dst.data_ptr(), B, H.data_ptr(), _stream(stream))
    return H


def hg_aca_bwd(src, dst, grad_H, want_src=True, want_dst=True, stream=None):
    """(grad_src, grad_dst), each shaped like src (or None when not wanted)."""
    B = _quad_rows(src, "src")
    _quad_rows(dst, "dst")
    _c(grad_H, "grad_H", torch.float64)
    gs = torch.empty_like(src) if want_src else None
    gd = torch.empty_like(dst) if want_dst else None
    _abi.call("hg_aca_bwd", src.data_ptr(), dst.data_ptr(), grad_H.data_ptr(), B,
              gs.data_ptr() if gs is not None else None,
              gd.data_ptr() if gd is not None else None, _stream(stream))
    return gs, gd


class ACAGeneral(torch.autograd.Function):
    """(src, dst) general quadrilaterals -> H (B, 9) float64 by ACA; backward
    by the hand-written reverse-mode kernel, to both point sets."""

    @staticmethod
    def forward(ctx, src, dst):
        src, dst = src.contiguous(), dst.contiguous()
        ctx.save_for_backward(src, dst)
        return hg_aca_fwd(src, dst)

    @staticmethod
    def backward(ctx, grad_H):
        src, dst = ctx.saved_tensors
        gs, gd = hg_aca_bwd(src, dst, grad_H.to(torch.float64).contiguous(),
                            ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        return gs, gd


def _img3(img, name):
    _c(img, name)
    if img.dim() != 3:
        raise ValueError(f"{name} must be (B, h, w)")
    return img.shape


def hg_warp_l1_fwd(H, img, tgt, stream=None):
    B, h, w = _img3(img, "img")
    _img3(tgt, "tgt")
    _c(H, "H", torch.float64)
    loss = torch.empty(B, dtype=torch.float32, device=img.device)
    _abi.call("hg_warp_l1_fwd", H.data_ptr(), img.data_ptr(), tgt.data_ptr(), B, h, w,
              loss.data_ptr(), _stream(stream))
    return loss


def hg_warp_l1_bwd(H, img, tgt, grad_loss, stream=None):
    B, h, w = _img3(img, "img")
    _img3(tgt, "tgt")
    _c(H, "H", torch.float64)
    _c(grad_loss, "grad_loss")
    gH = torch.empty((B, 9), dtype=torch.float64, device=img.device)
    _abi.call("hg_warp_l1_bwd", H.data_ptr(), img.data_ptr(), tgt.data_ptr(),
              grad_loss.data_ptr(), B, h, w, gH.data_ptr(), _stream(stream))
    return gH


def hg_warp_store_fwd(H, img, stream=None):
    B, h, w = _img3(img, "img")
    out = torch.empty_like(img)
    _abi.call("hg_warp_store_fwd", _c(H, "H", torch.float64).data_ptr(), img.data_ptr(), B, h, w,
              out.data_ptr(), _stream(stream))
    return out


def hg_l1_fwd(warped, tgt, stream=None):
    B, h, w = _img3(warped, "warped")
    _img3(tgt, "tgt")
    loss = torch.empty(B, dtype=torch.float32, device=warped.device)
    _abi.call("hg_l1_fwd", warped.data_ptr(), tgt.data_ptr(), B, h, w, loss.data_ptr(),
              _stream(stream))
    return loss


def hg_l1_bwd(warped, tgt, grad_loss, stream=None):
    B, h, w = _img3(warped, "warped")
    g = torch.empty_like(warped)
    _abi.call("hg_l1_bwd", warped.data_ptr(), _c(tgt, "tgt").data_ptr(),
              _c(grad_loss, "grad_loss").data_ptr(), B, h, w, g.data_ptr(), _stream(stream))
    return g


def hg_warp_bwd_from_grad(H, img, grad_warped, stream=None):
    B, h, w = _img3(img, "img")
    gH = torch.empty((B, 9), dtype=torch.float64, device=img.device)
    _abi.call("hg_warp_bwd_from_grad", _c(H, "H", torch.float64).data_ptr(), img.data_ptr(),
              _c(grad_warped, "grad_warped").data_ptr(), B, h, w, gH.data_ptr(), _stream(stream))
    return gH


class ACARect(torch.autograd.Function):
    """offsets (B, 4, 2) float32 -> H (B, 9) float64 by ACA with the source
    corners at the rectangle's; backward by the hand-written reverse-mode
    kernel."""

    @staticmethod
    def forward(ctx, offsets, x0, y0, w, r):
        offsets = offsets.contiguous()
        ctx.save_for_backward(offsets)
        ctx.rect = (x0, y0, w, r)
        return hg_aca_rect_fwd(offsets, x0, y0, w, r)

    @staticmethod
    def backward(ctx, grad_H):
        (offsets,) = ctx.saved_tensors
        g = hg_aca_rect_bwd(offsets, grad_H.to(torch.float64).contiguous(), *ctx.rect)
        return g, None, None, None, None


class WarpL1(torch.autograd.Function):
    """(H, img, tgt) -> per-patch L1 loss of the warp; the backward recomputes
    every per-pixel quantity from H (nothing per pixel is saved)."""

    @staticmethod
    def forward(ctx, H, img, tgt):
        H, img, tgt = H.contiguous(), img.contiguous(), tgt.contiguous()
        ctx.save_for_backward(H, img, tgt)
        return hg_warp_l1_fwd(H, img, tgt)

    @staticmethod
    def backward(ctx, grad_loss):
        H, img, tgt = ctx.saved_tensors
        gl = grad_loss.to(torch.float32).contiguous()
        return hg_warp_l1_bwd(H, img, tgt, gl), None, None


def hg_photometric_fwd(offsets, img, tgt, stream=None):
    """Fused offsets (B, 4, 2) -> per-patch loss (B,) (ACA + warp + L1)."""
    _c(offsets, "offsets")
    B, h, w = _img3(img, "img")
    _img3(tgt, "tgt")
    loss = torch.empty(B, dtype=torch.float32, device=img.device)
    _abi.call("hg_photometric_fwd", offsets.data_ptr(), img.data_ptr(), tgt.data_ptr(), B, h, w,
              loss.data_ptr(), _stream(stream))
    return loss


def hg_photometric_bwd(offsets, img, tgt, grad_loss, stream=None):
    """Fused gradient: grad_loss[b] * dloss_b/d offsets_b, (B, 4, 2) float32."""
    _c(offsets, "offsets")
    B, h, w = _img3(img, "img")
    _img3(tgt, "tgt")
    _c(grad_loss, "grad_loss")
    g = torch.empty((B, 4, 2), dtype=torch.float32, device=img.device)
    _abi.call("hg_photometric_bwd", offsets.data_ptr(), img.data_ptr(), tgt.data_ptr(),
              grad_loss.data_ptr(), B, h, w, g.data_ptr(), _stream(stream))
    return g


def hg_photometric_fwd_grad(offsets, img, tgt, stream=None):
    """Loss and its gradient in one pass: (loss (B,), grad_unit (B, 4, 2)) with
    grad_unit[b] = dloss_b/d offsets_b."""
    _c(offsets, "offsets")
    B, h, w = _img3(img, "img")
    _img3(tgt, "tgt")
    loss = torch.empty(B, dtype=torch.float32, device=img.device)
    g = torch.empty((B, 4, 2), dtype=torch.float32, device=img.device)
    _abi.call("hg_photometric_fwd_grad", offsets.data_ptr(), img.data_ptr(), tgt.data_ptr(), B, h,
              w, loss.data_ptr(), g.data_ptr(), _stream(stream))
    return loss, g


def hg_scale_grad(grad_unit, grad_loss, stream=None):
    """grad_loss[b] * grad_unit[b] for (B, 4, 2) grad_unit, (B,) grad_loss."""
    _c(grad_unit, "grad_unit")
    _c(grad_loss, "grad_loss")
    B = grad_unit.shape[0]
    if tuple(grad_unit.shape) != (B, 4, 2) or grad_loss.numel() != B:
        raise ValueError("grad_unit must be (B, 4, 2) and grad_loss (B,)")
    out = torch.empty_like(grad_unit)
    _abi.call("hg_scale_grad", grad_unit.data_ptr(), grad_loss.data_ptr(), B, out.data_ptr(),
              _stream(stream))
    return out


class PhotometricL1(torch.autograd.Function):
    """offsets -> per-patch loss. When the offsets need a gradient, one launch
    computes the loss and its gradient together (img and tgt are read once;
    8 floats per patch are kept) and the backward scales that gradient by
    grad_loss; otherwise a loss-only launch."""

    @staticmethod
    def forward(ctx, offsets, img, tgt):
        offsets, img, tgt = offsets.contiguous(), img.contiguous(), tgt.contiguous()
        if ctx.needs_input_grad[0]:
            loss, g = hg_photometric_fwd_grad(offsets, img, tgt)
            ctx.save_for_backward(g)
            return loss
        return hg_photometric_fwd(offsets, img, tgt)

    @staticmethod
    def backward(ctx, grad_loss):
        (g,) = ctx.saved_tensors
        gl = grad_loss.to(torch.float32).contiguous()
        return hg_scale_grad(g, gl), None, None


class PhotometricL1Recompute(torch.autograd.Function):
    """offsets -> per-patch loss in one fused launch; backward in one fused
    launch that recomputes H, the warp and ACA's reverse mode (nothing per
    patch is kept but the inputs)."""

    @staticmethod
    def forward(ctx, offsets, img, tgt):
        offsets, img, tgt = offsets.contiguous(), img.contiguous(), tgt.contiguous()
        ctx.save_for_backward(offsets, img, tgt)
        return hg_photometric_fwd(offsets, img, tgt)

    @staticmethod
    def backward(ctx, grad_loss):
        offsets, img, tgt = ctx.saved_tensors
        gl = grad_loss.to(torch.float32).contiguous()
        return hg_photometric_bwd(offsets, img, tgt, gl), None, None


def photometric_loss(offsets, img, tgt, fused=True):
    """Per-patch loss of the 4-point-offset pipeline for h x w patches with
    corners at the pixel centres (0, 0) .. (w-1, h-1); differentiable in
    offsets. ``fused=True``: single-pass loss and gradient (PhotometricL1);
    ``"recompute"``: fused forward and recomputing backward launches;
    ``False``: the separate ACARect and WarpL1 stages (same arithmetic)."""
    if fused == "recompute":
        return PhotometricL1Recompute.apply(offsets, img, tgt)
    if fused:
        return PhotometricL1.apply(offsets, img, tgt)
    h, w = img.shape[-2:]
    H = ACARect.apply(offsets, 0.0, 0.0, float(w - 1), float(w - 1) / float(h - 1))
    return WarpL1.apply(H, img, tgt)


class Refine:
    """Iterative refinement of 4-point offsets (hg_refine): ``iters`` rounds
    of ACA -> warp + L1 backward -> reverse mode -> offsets -= step *
    grad on h x w patches (one fused launch per iteration); ``run()`` launches eagerly,
    ``graph()`` captures the same sequence for replay. ``offsets`` (B, 4, 2)
    float32 is updated in place; ``loss`` (B,) holds the final loss."""

    def __init__(self, img, tgt, offsets, iters=6, step=1.0, with_loss=True):
        _img3(img, "img")
        _img3(tgt, "tgt")
        self.img, self.tgt = img, tgt
        self.offsets = _c(offsets, "offsets")
        self.B, self.h, self.w = img.shape
        if tuple(offsets.shape) != (self.B, 4, 2) or tuple(tgt.shape) != tuple(img.shape):
            raise ValueError("shapes: img, tgt (B, h, w); offsets (B, 4, 2)")
        self.iters, self.step = int(iters), float(step)
        self.loss = torch.empty(self.B, dtype=torch.float32, device=img.device) if with_loss else None

    def _args(self):
        return (self.img.data_ptr(), self.tgt.data_ptr(), self.B, self.h, self.w, self.iters,
                self.step, self.offsets.data_ptr(),
                self.loss.data_ptr() if self.loss is not None else None)

    def run(self, stream=None):
        _abi.call("hg_refine", *self._args(), _stream(stream))
        return self.offsets, self.loss

    def graph(self, stream=None):
        h = C.c_void_p()
        _abi.call("hg_refine_graph_create", *self._args(), _stream(stream), C.byref(h))
        return Graph(h, self)
