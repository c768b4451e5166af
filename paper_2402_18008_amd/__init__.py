"""MI355X-native minimal 4-point homography (ACA / SKS) with fused RANSAC
scoring and a differentiable 4-point-offset pipeline.

Thin torch binding over libhomog (include/homog.h): every function marshals
device tensors into the C ABI on the current HIP stream; all computation runs
in the library's HIP kernels. Function names match the C entry points.
"""
from __future__ import annotations

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
