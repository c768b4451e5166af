"""4-point-offset pipeline reference in torch float64 on the CPU (oracle; test
infrastructure only).

The deep-homography use of the solver (Sec. 5.3 and the deep pipeline
experiments): four corner offsets of a square source patch define the target
quadrilateral; the homography between them warps the image; a photometric L1
loss compares the warp with a target patch; gradients flow back to the offsets.

Conventions of this implementation (the paper fixes none of them):

* source corners of an S x S patch are the pixel centres (0, 0), (S-1, 0),
  (S-1, S-1), (0, S-1), in the order TL, TR, BR, BL (= M, N, Q, P), and the
  target corners are those plus the offsets;
* H maps source corners to target corners; the warp samples the source image
  at pi(H^-1 p) for every pixel p = (x, y) of the output (x = column);
* bilinear interpolation with x0 = floor(x); taps outside the image read 0;
* loss per patch L_b = mean_p |I_w(p) - T(p)|; gradients follow torch autograd
  (sign(0) = 0, floor has zero derivative).

Here H is the plain definition (DLT with h33 = 1 solved by
``torch.linalg.solve``) and H^-1 comes from ``torch.linalg.inv``; autograd runs
through both.
"""
from __future__ import annotations

import torch

from . import homography as hg


def square_corners(size, dtype=torch.float64):
    """Corners TL, TR, BR, BL of a size x size patch, or of an h x w patch when
    ``size`` is a pair (h, w)."""
    h, w = (size, size) if isinstance(size, int) else size
    a, b = float(w - 1), float(h - 1)
    return torch.tensor([[0.0, 0.0], [a, 0.0], [a, b], [0.0, b]], dtype=dtype)


def h_dlt(offsets, size):
    """H (B, 3, 3) with h33 = 1 mapping the square's corners to corners +
    offsets (B, 4, 2), by solving the 8x8 DLT system."""
    src = square_corners(size, offsets.dtype)
    dst = src[None] + offsets
    B = offsets.shape[0]
    A = offsets.new_zeros(B, 8, 8)
    b = offsets.new_zeros(B, 8)
    for k in range(4):
        x, y = src[k, 0], src[k, 1]
        u, v = dst[:, k, 0], dst[:, k, 1]
        r = 2 * k
        A[:, r, 0] = x
        A[:, r, 1] = y
        A[:, r, 2] = 1.0
        A[:, r, 6] = -u * x
        A[:, r, 7] = -u * y
        b[:, r] = u
        A[:, r + 1, 3] = x
        A[:, r + 1, 4] = y
        A[:, r + 1, 5] = 1.0
        A[:, r + 1, 6] = -v * x
        A[:, r + 1, 7] = -v * y
        b[:, r + 1] = v
    h = torch.linalg.solve(A, b)
    return torch.cat([h, offsets.new_ones(B, 1)], dim=1).reshape(B, 3, 3)


def h_rect(offsets, size):
    """H from Algorithm 1 (rectangle with corners at the pixel centres: x0 =
    y0 = 0, width w-1, aspect (w-1)/(h-1)) on torch tensors; autograd gives
    its Jacobian."""
    src = square_corners(size, offsets.dtype)
    dst = src[None] + offsets
    # Algorithm 1 takes M N P Q = TL TR BL BR
    M, N, Q, P = dst[:, 0], dst[:, 1], dst[:, 2], dst[:, 3]
    q = [M[:, 0], M[:, 1], N[:, 0], N[:, 1], P[:, 0], P[:, 1], Q[:, 0], Q[:, 1]]
    wr, hr = float(src[1, 0]), float(src[2, 1])
    H = hg.aca_rect_s(0.0, 0.0, wr, wr / hr, q, square=(wr == hr))
    return torch.stack([torch.stack(r, dim=-1) for r in H], dim=-2)


def h_aca(src, dst):
    """General ACA (Sec. 4, the structured order of ``homography.aca_s``) on
    torch tensors: src, dst (B, 8) as x_M y_M x_N y_N x_P y_P x_Q y_Q; returns
    H (B, 3, 3) at ACA's own scale. Autograd through it gives the reverse mode
    of the tensorised general solver."""
    H = hg.aca_s(list(src.T), list(dst.T))
    return torch.stack([torch.stack(r, dim=-1) for r in H], dim=-2)


def h_aca_poly(src, dst):
    """General ACA through its polynomial form (Sec. 4.5, eq. H_11, with the
    third-column reading of ``homography.aca_poly_s``) on torch tensors, src,
    dst (B, 8); H (B, 3, 3) at the same scale as ``h_aca``. Autograd through it
    differentiates the nine polynomials of the corner coordinates directly."""
    H = hg.aca_poly_s(list(src.T), list(dst.T))
    return torch.stack([torch.stack(r, dim=-1) for r in H], dim=-2)


def aca_poly_vjp(src, dst, grad_H):
    """(dH/dsrc)^T grad_H and (dH/ddst)^T grad_H, each (B, 8), for H = h_aca_poly
    and grad_H (B, 3, 3), by float64 autograd through the polynomial form."""
    s = torch.as_tensor(src, dtype=torch.float64).clone().requires_grad_(True)
    d = torch.as_tensor(dst, dtype=torch.float64).clone().requires_grad_(True)
    g = torch.as_tensor(grad_H, dtype=torch.float64)
    H = h_aca_poly(s, d)
    gs, gd = torch.autograd.grad((H * g).sum(), (s, d))
    return gs, gd


def aca_vjp(src, dst, grad_H):
    """(dH/dsrc)^T grad_H and (dH/ddst)^T grad_H, each (B, 8), for H = h_aca
    and grad_H (B, 3, 3), by float64 autograd."""
    s = torch.as_tensor(src, dtype=torch.float64).clone().requires_grad_(True)
    d = torch.as_tensor(dst, dtype=torch.float64).clone().requires_grad_(True)
    g = torch.as_tensor(grad_H, dtype=torch.float64)
    H = h_aca(s, d)
    gs, gd = torch.autograd.grad((H * g).sum(), (s, d))
    return gs, gd


def bilinear_zero(img, sx, sy):
    """Sample img (B, h, w) at (sx, sy) (B, P) with zero padding."""
    B, h, w = img.shape
    x0 = torch.floor(sx)
    y0 = torch.floor(sy)
    ax = sx - x0
    ay = sy - y0
    flat = img.reshape(B, h * w)
    out = 0.0
    for dy, wy in ((0, 1 - ay), (1, ay)):
        for dx, wx in ((0, 1 - ax), (1, ax)):
            xi = (x0 + dx).long()
            yi = (y0 + dy).long()
            inside = (xi >= 0) & (xi < w) & (yi >= 0) & (yi < h)
            lin = torch.where(inside, yi * w + xi, torch.zeros_like(xi))
            val = torch.gather(flat, 1, lin) * inside.to(img.dtype)
            out = out + wx * wy * val
    return out


def warp(img, H):
    """Source image (B, h, w) warped into the target frame: I(pi(H^-1 p))."""
    B, h, w = img.shape
    G = torch.linalg.inv(H)
    ys, xs = torch.meshgrid(torch.arange(h, dtype=H.dtype), torch.arange(w, dtype=H.dtype),
                            indexing="ij")
    p = torch.stack([xs.reshape(-1), ys.reshape(-1), torch.ones(h * w, dtype=H.dtype)])
    q = G @ p                                       # (B, 3, P)
    sx = q[:, 0] / q[:, 2]
    sy = q[:, 1] / q[:, 2]
    return bilinear_zero(img, sx, sy).reshape(B, h, w)


def loss(offsets, img, tgt, solver=h_dlt):
    """Per-patch loss (B,) = mean |warp(img, H(offsets)) - tgt|."""
    H = solver(offsets, tuple(img.shape[-2:]))
    return (warp(img, H) - tgt).abs().mean(dim=(1, 2))


def loss_and_grad(offsets, img, tgt, solver=h_dlt, chunk=64):
    """Loss (B,) and dL_b/d offsets_b (B, 4, 2) by float64 autograd, in chunks."""
    off = torch.as_tensor(offsets, dtype=torch.float64)
    im = torch.as_tensor(img, dtype=torch.float64)
    tg = torch.as_tensor(tgt, dtype=torch.float64)
    Ls, Gs = [], []
    for a in range(0, off.shape[0], chunk):
        o = off[a:a + chunk].clone().requires_grad_(True)
        L = loss(o, im[a:a + chunk], tg[a:a + chunk], solver)
        (g,) = torch.autograd.grad(L.sum(), o)
        Ls.append(L.detach())
        Gs.append(g)
    return torch.cat(Ls), torch.cat(Gs)


def loss_fd_grad(offsets, img, tgt, h=1e-6, solver=h_dlt):
    """Central finite-difference gradient of each patch's loss (B, 4, 2)."""
    off = torch.as_tensor(offsets, dtype=torch.float64)
    im = torch.as_tensor(img, dtype=torch.float64)
    tg = torch.as_tensor(tgt, dtype=torch.float64)
    g = torch.zeros_like(off)
    with torch.no_grad():
        for k in range(4):
            for c in range(2):
                e = torch.zeros_like(off)
                e[:, k, c] = h
                g[:, k, c] = (loss(off + e, im, tg, solver) - loss(off - e, im, tg, solver)) / (2 * h)
    return g


def refine_ref(offsets, img, tgt, iters, step, solver=h_dlt):
    """Iterative refinement of float32 offsets (B, 4, 2): each iteration takes
    every patch's float64 loss gradient at the current offsets, rounds it to
    float32 and sets offsets = offsets - step * gradient in float32 (the
    network's predicted update of an iterative deep homography pipeline
    replaced by a gradient step). Returns (offsets float32, loss float64 at
    the final offsets)."""
    import numpy as np
    off = np.array(offsets, dtype=np.float32, copy=True)
    st = np.float32(step)
    for _ in range(iters):
        _, g = loss_and_grad(off.astype(np.float64), img, tgt, solver)
        off = off - st * g.numpy().astype(np.float32)
    L = loss(torch.as_tensor(off, dtype=torch.float64), torch.as_tensor(img, dtype=torch.float64),
             torch.as_tensor(tgt, dtype=torch.float64), solver)
    return off, L.detach()
