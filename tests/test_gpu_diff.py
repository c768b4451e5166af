"""Differentiable 4-point-offset pipeline on the GPU against the float64 oracle.

Per-patch steps (H, G = adj H, the sample position and the floor that picks
the bilinear cell) are double precision; the per-pixel terms after the floor
(bilinear weights, taps, residual, gradient terms) are float with double
per-patch sums. Bars: H within 1e-12 (Frobenius-normalised) of the oracle's;
its vector-Jacobian product within 1e-6 relative (float output); per-patch
loss within 1e-6 relative; the per-patch gradient with respect to the 8
offsets within GRAD_TOL = 1e-4 relative (norm-wise) of float64 autograd
through the DLT solve (float sums over h w terms with sign cancellation), the
error distribution printed. Float64 central finite differences (h = 1e-6)
agree within FD_TOL. The single-pass (loss and gradient together),
recomputing and separate-stage forms agree within 1e-6 (loss) and 1e-5
(gradient: their sums run in different orders); the
stored-intermediate form rounds nothing that the others do not, and agrees
within 1e-5."""
import numpy as np
import pytest
import torch

import synth
from oracle import homography as hg
from oracle import warp as ow
from tests.gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu
GRAD_TOL = 1e-4
FD_TOL = 1e-4


def rel(a, b):
    a = np.asarray(a, np.float64).reshape(len(a), -1)
    b = np.asarray(b, np.float64).reshape(len(b), -1)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


def rect_src_dst(off, x0, y0, w, r):
    """Source (M N P Q = TL TR BL BR) of the rectangle and the targets
    corners + offsets (offset order TL TR BR BL), as (B, 8) float64."""
    s = np.array(hg.rect_corners(x0, y0, w, r), np.float64)   # M N P Q
    o = off.astype(np.float64).reshape(-1, 4, 2)[:, [0, 1, 3, 2], :].reshape(-1, 8)
    return np.broadcast_to(s, o.shape).copy(), s[None] + o


def test_rect_forward_backward():
    """The rectangle H is ACA's with the rectangle's source corners: raw
    values within 1e-12 of the oracle's general ACA, equal up to scale to
    Algorithm 1 and to the exact solution; its vector-Jacobian product is the
    oracle's (float64 autograd through general ACA, through its polynomial
    form and through Algorithm 1)."""
    require_gpu()
    import paper_2402_18008_amd as hgpu
    rng = np.random.default_rng(0)
    off = rng.uniform(-32, 32, (300, 4, 2)).astype(np.float32)
    announce("aca_rect fwd/bwd B=300")
    H = hgpu.hg_aca_rect_fwd(torch.from_numpy(off).cuda(), 0.0, 0.0, 127.0, 1.0).cpu().numpy()
    src, dst = rect_src_dst(off, 0.0, 0.0, 127.0, 1.0)
    d64 = torch.from_numpy(dst).requires_grad_(True)
    Ha = ow.h_aca(torch.from_numpy(src), d64)
    assert np.abs(H.reshape(-1, 3, 3) - Ha.detach().numpy()).max() / np.abs(Ha.detach().numpy()).max() < 1e-12
    o64 = torch.from_numpy(off.astype(np.float64)).requires_grad_(True)
    Hr = ow.h_rect(o64, 128)
    assert hg.herr(H.reshape(-1, 3, 3), Hr.detach().numpy()).max() < 1e-12
    gH = rng.normal(size=(300, 9))
    g = hgpu.hg_aca_rect_bwd(torch.from_numpy(off).cuda(), torch.from_numpy(gH).cuda(), 0.0, 0.0,
                             127.0, 1.0).cpu().numpy()
    (gd,) = torch.autograd.grad((Ha * torch.from_numpy(gH).reshape(-1, 3, 3)).sum(), d64,
                                retain_graph=True)
    gref = gd.numpy().reshape(-1, 4, 2)[:, [0, 1, 3, 2], :]      # back to TL TR BR BL
    assert rel(g, gref).max() < 1e-6     # float output
    # d(H)/d(offsets) through ACA's polynomial form (eq. H_11) gives the same products
    _, gdp = ow.aca_poly_vjp(torch.from_numpy(src), torch.from_numpy(dst),
                             torch.from_numpy(gH).reshape(-1, 3, 3))
    assert rel(g, gdp.numpy().reshape(-1, 4, 2)[:, [0, 1, 3, 2], :]).max() < 1e-6
    # the same direction through Algorithm 1: H differs by a per-patch scale
    # s(offsets), so grad_H projected orthogonally to H gives equal products
    Hn = Ha.detach().numpy().reshape(-1, 9)
    Hn = Hn / np.linalg.norm(Hn, axis=1, keepdims=True)
    gperp = gH - (gH * Hn).sum(1, keepdims=True) * Hn
    gp = hgpu.hg_aca_rect_bwd(torch.from_numpy(off).cuda(), torch.from_numpy(gperp).cuda(), 0.0,
                              0.0, 127.0, 1.0).cpu().numpy()
    Ha_n = Ha / Ha.reshape(-1, 9).norm(dim=1)[:, None, None]
    Hr_n = Hr / Hr.reshape(-1, 9).norm(dim=1)[:, None, None] * torch.sign(
        (Hr * Ha).reshape(-1, 9).sum(1))[:, None, None]
    (ga,) = torch.autograd.grad((Ha_n * torch.from_numpy(gperp).reshape(-1, 3, 3)).sum(), d64)
    (gr,) = torch.autograd.grad((Hr_n * torch.from_numpy(gperp).reshape(-1, 3, 3)).sum(), o64)
    ga = ga.numpy().reshape(-1, 4, 2)[:, [0, 1, 3, 2], :]
    assert rel(ga, gr.numpy()).max() < 1e-9      # normalised H: same function of offsets
    # a general rectangle (x0, y0, w, r)
    x0, y0, w, r = 3.0, -2.0, 50.0, 1.25
    H = hgpu.hg_aca_rect_fwd(torch.from_numpy(off).cuda(), x0, y0, w, r).cpu().numpy()
    src = hg.rect_corners(x0, y0, w, r)
    for b in range(0, 300, 37):
        d = off[b].astype(np.float64)
        dst = [src[0] + d[0, 0], src[1] + d[0, 1], src[2] + d[1, 0], src[3] + d[1, 1],
               src[4] + d[3, 0], src[5] + d[3, 1], src[6] + d[2, 0], src[7] + d[2, 1]]
        Hx = hg.exact_h(src, dst)
        assert hg.herr(H[b].reshape(3, 3), Hx) < 1e-12


def run_pipeline(pb, idx=None, fused=True):
    import paper_2402_18008_amd as hgpu
    sel = slice(None) if idx is None else idx
    off = torch.from_numpy(pb.offsets[sel]).cuda().requires_grad_(True)
    img = torch.from_numpy(pb.img[sel]).cuda()
    tgt = torch.from_numpy(pb.tgt[sel]).cuda()
    L = hgpu.photometric_loss(off, img, tgt, fused=fused)
    (g,) = torch.autograd.grad(L.sum(), off)
    torch.cuda.synchronize()
    return L.detach().cpu().numpy(), g.cpu().numpy()


def compare_oracle(pb, L, g, idx, label):
    Lr, gr = ow.loss_and_grad(pb.offsets[idx], pb.img[idx], pb.tgt[idx])
    el = np.abs(L - Lr.numpy()) / np.abs(Lr.numpy())
    eg = rel(g, gr.numpy())
    print(f"{label}: loss rel err max {el.max():.2e}; grad rel err median {np.median(eg):.2e} "
          f"p90 {np.quantile(eg, 0.9):.2e} max {eg.max():.2e}")
    assert el.max() < 1e-6, label
    assert eg.max() < GRAD_TOL, label
    return el, eg


@pytest.mark.parametrize("fused", [True, "recompute", False])
def test_small_patches_against_oracle(fused):
    require_gpu()
    pb = synth.patches(24, 21, size=64, sigma=3.0, max_shift=8, max_offset=12.0)
    announce(f"warp-l1 fwd+bwd 24 patches 64x64 fused={fused}")
    L, g = run_pipeline(pb, fused=fused)
    compare_oracle(pb, L, g, slice(None), "64x64")
    # finite differences of the float64 oracle agree with the same gradient
    fd = ow.loss_fd_grad(pb.offsets[:4], pb.img[:4], pb.tgt[:4], h=1e-6).numpy()
    assert rel(g[:4], fd).max() < FD_TOL


def test_other_patch_sizes():
    """Sizes other than the benchmark's: 150 x 140 and 33 x 45 (w not a
    multiple of 4), fused and separate stages, against the oracle."""
    require_gpu()
    for B, h, w, seed in ((3, 150, 140, 31), (4, 33, 45, 32)):
        rng = np.random.default_rng(seed)
        pbl = type("PB", (), {})()
        pbl.img = rng.normal(size=(B, h, w)).astype(np.float32)
        pbl.tgt = rng.normal(size=(B, h, w)).astype(np.float32)
        pbl.offsets = rng.uniform(-6, 6, (B, 4, 2)).astype(np.float32)
        announce(f"warp-l1 fwd+bwd {B} patches {h}x{w}")
        for fused in (True, False):
            L, g = run_pipeline(pbl, fused=fused)
            compare_oracle(pbl, L, g, slice(None), f"{h}x{w} fused={fused}")


@pytest.mark.parametrize("fused", [True, "recompute", False])
def test_tiny_patches_one_partial_iteration(fused):
    """Patches smaller than one iteration of the pixel loop (every pixel lies
    in the masked last iteration) and widths of 2 (one column pair spans the
    row), against the oracle."""
    require_gpu()
    for B, h, w, seed in ((3, 2, 2, 51), (4, 3, 5, 52), (2, 8, 8, 53), (2, 5, 2, 54)):
        rng = np.random.default_rng(seed)
        pbl = type("PB", (), {})()
        pbl.img = rng.normal(size=(B, h, w)).astype(np.float32)
        pbl.tgt = rng.normal(size=(B, h, w)).astype(np.float32)
        pbl.offsets = rng.uniform(-0.4, 0.4, (B, 4, 2)).astype(np.float32)
        announce(f"warp-l1 fwd+bwd {B} patches {h}x{w} fused={fused}")
        L, g = run_pipeline(pbl, fused=fused)
        compare_oracle(pbl, L, g, slice(None), f"{h}x{w} fused={fused}")


def test_one_pixel_wide_images():
    """w = 1 (the warp kernels accept it): a tap's column pair then reaches
    into the next row, and past the buffer's end on the last row. The stored
    warp equals the oracle's for the identity and for a small shift."""
    require_gpu()
    import paper_2402_18008_amd as hgpu
    rng = np.random.default_rng(61)
    B, h, w = 3, 9, 1
    img = torch.from_numpy(rng.normal(size=(B, h, w)).astype(np.float32)).cuda()
    for dy in (0.0, 0.3, -0.7):
        Hd = torch.eye(3, dtype=torch.float64).repeat(B, 1, 1)
        Hd[:, 1, 2] = dy
        announce(f"warp w=1 dy={dy}")
        Wp = hgpu.hg_warp_store_fwd(Hd.reshape(B, 9).cuda(), img)
        torch.cuda.synchronize()
        Wr = ow.warp(img.double().cpu(), Hd)
        assert (Wr - Wp.double().cpu()).abs().max() < 4e-6, dy
        if dy == 0.0:
            assert torch.equal(Wp.cpu(), img.cpu())


def test_warp_and_gradient_over_image_shapes():
    """Random perspective maps that move parts of the patch outside the image,
    over image shapes from 1 x 1 up: widths that divide the workgroup (each
    thread walks one column) and that do not, widths wider than a workgroup,
    one-pixel rows and columns. The stored warp equals the oracle's warp, and on
    every shape the L1 loss and its gradient with respect to H match float64
    autograd through the oracle's warp."""
    require_gpu()
    import paper_2402_18008_amd as hgpu
    rng = np.random.default_rng(73)
    shapes = [(1, 1), (1, 7), (7, 1), (2, 2), (3, 5), (16, 16), (17, 33), (64, 3), (5, 300),
              (40, 257), (33, 64), (128, 128), (9, 512), (300, 2)]
    for h, w in shapes:
        B = 3
        img = torch.from_numpy(rng.normal(size=(B, h, w)).astype(np.float32))
        tgt = torch.from_numpy(rng.normal(size=(B, h, w)).astype(np.float32))
        Hd = torch.zeros(B, 3, 3, dtype=torch.float64)
        for b in range(B):
            s_ = max(h, w)
            Hd[b] = torch.tensor([[1 + 0.1 * rng.uniform(-1, 1), 0.1 * rng.uniform(-1, 1),
                                   w * rng.uniform(-0.4, 0.4)],
                                  [0.1 * rng.uniform(-1, 1), 1 + 0.1 * rng.uniform(-1, 1),
                                   h * rng.uniform(-0.4, 0.4)],
                                  [rng.uniform(-1, 1) * 0.02 / s_, rng.uniform(-1, 1) * 0.02 / s_, 1.0]],
                                 dtype=torch.float64)
        announce(f"warp and L1 gradient {h}x{w}")
        Hc = Hd.reshape(B, 9).cuda()
        Wp = hgpu.hg_warp_store_fwd(Hc, img.cuda())
        L = hgpu.hg_warp_l1_fwd(Hc, img.cuda(), tgt.cuda())
        gH = hgpu.hg_warp_l1_bwd(Hc, img.cuda(), tgt.cuda(), torch.ones(B, device="cuda"))
        torch.cuda.synchronize()
        Wr = ow.warp(img.double(), Hd)
        assert (Wr - Wp.double().cpu()).abs().max() < 4e-6, (h, w)
        Hr = Hd.clone().requires_grad_(True)
        Lr = (ow.warp(img.double(), Hr) - tgt.double()).abs().mean(dim=(1, 2))
        (gr,) = torch.autograd.grad(Lr.sum(), Hr)
        assert np.allclose(L.cpu().numpy(), Lr.detach().numpy(), rtol=1e-5, atol=1e-7), (h, w)
        eg = rel(gH.cpu().numpy().reshape(B, 9), gr.numpy().reshape(B, 9))
        assert eg.max() < GRAD_TOL, (h, w, eg.max())


def test_batch_of_several_rounds():
    """4096 patches of 64 x 64: about four rounds of resident workgroups (the
    per-wave priority schedule restarts in each); the single pass, the two
    passes and the separate stages agree on every patch, and 16 sampled
    patches match the oracle."""
    require_gpu()
    pb = synth.patches(4096, 29, size=64, sigma=3.0, max_shift=8, max_offset=12.0)
    announce("warp-l1 fwd+bwd 4096 patches 64x64, three forms")
    L1, g1 = run_pipeline(pb, fused=True)
    for form in ("recompute", False):
        L2, g2 = run_pipeline(pb, fused=form)
        assert np.allclose(L1, L2, rtol=1e-6, atol=0), form
        assert rel(g1, g2).max() < 1e-5, form
    idx = np.arange(0, 4096, 256)
    compare_oracle(pb, L1[idx], g1[idx], idx, "4096 patches, sampled")


def test_ragged_sizes_and_stored_form():
    require_gpu()
    import paper_2402_18008_amd as hgpu
    rng = np.random.default_rng(3)
    B, h, w = 5, 37, 53
    img = torch.from_numpy(rng.normal(size=(B, h, w)).astype(np.float32)).cuda()
    tgt = torch.from_numpy(rng.normal(size=(B, h, w)).astype(np.float32)).cuda()
    off = torch.from_numpy(rng.uniform(-5, 5, (B, 4, 2)).astype(np.float32)).cuda()
    announce("warp-l1 ragged 37x53, stored vs recompute")
    H = hgpu.hg_aca_rect_fwd(off, 0.0, 0.0, float(w - 1), float(w - 1) / float(h - 1))
    L = hgpu.hg_warp_l1_fwd(H, img, tgt)
    Wp = hgpu.hg_warp_store_fwd(H, img)
    L2 = hgpu.hg_l1_fwd(Wp, tgt)
    gl = torch.rand(B, device="cuda")
    gH = hgpu.hg_warp_l1_bwd(H, img, tgt, gl)
    gW = hgpu.hg_l1_bwd(Wp, tgt, gl)
    gH2 = hgpu.hg_warp_bwd_from_grad(H, img, gW)
    torch.cuda.synchronize()
    assert torch.allclose(L, L2, rtol=1e-6, atol=0)
    assert rel(gH.cpu().numpy(), gH2.cpu().numpy()).max() < 1e-5
    # against the oracle's warp of the same H
    Hd = H.cpu().reshape(B, 3, 3)
    Wr = ow.warp(img.double().cpu(), Hd)
    # (float bilinear evaluation: a few float ulps of values up to ~5)
    assert (Wr - Wp.double().cpu()).abs().max() < 4e-6
    # and the whole pipeline against the oracle's autograd
    pbl = type("PB", (), {})()
    pbl.offsets, pbl.img, pbl.tgt = off.cpu().numpy(), img.cpu().numpy(), tgt.cpu().numpy()
    Lg, gg = run_pipeline(pbl)
    compare_oracle(pbl, Lg, gg, slice(None), "37x53")
    # zero offsets: the warp is the identity
    H0 = hgpu.hg_aca_rect_fwd(torch.zeros_like(off), 0.0, 0.0, float(w - 1), float(w - 1) / float(h - 1))
    W0 = hgpu.hg_warp_store_fwd(H0, img)
    assert (W0 - img).abs().max() < 1e-6
    # empty batch
    z = torch.empty((0, h, w), device="cuda")
    assert hgpu.hg_warp_l1_fwd(torch.empty((0, 9), dtype=torch.float64, device="cuda"), z, z).numel() == 0


def test_config4_full_batch_sampled():
    """B = 1024 patches of 128 x 128 in one call (single-pass and recomputing
    forms); 32 sampled patches against float64 autograd through the DLT solve
    and 4 against float64 central finite differences."""
    require_gpu()
    announce("warp-l1 config4 B=1024 generating")
    pb = synth.config4()
    announce("warp-l1 config4 fwd+bwd")
    L, g = run_pipeline(pb)
    Lr, gr = run_pipeline(pb, fused="recompute")
    assert np.isfinite(L).all() and np.isfinite(g).all()
    # (the two forms run with different workgroup sizes, so their sums differ in order)
    assert np.allclose(L, Lr, rtol=1e-6, atol=0) and rel(g, gr).max() < 1e-6
    idx = np.random.default_rng(1).choice(1024, 32, replace=False)
    compare_oracle(pb, L[idx], g[idx], idx, "config4")
    fd_idx = idx[:4]
    fd = ow.loss_fd_grad(pb.offsets[fd_idx], pb.img[fd_idx], pb.tgt[fd_idx], h=1e-6).numpy()
    efd = rel(g[fd_idx], fd)
    print("config4 finite differences: rel err", efd)
    assert efd.max() < FD_TOL


@pytest.mark.parametrize("B", [1, 3, 257, 1000])
def test_general_aca_forward_backward(B):
    """General quadrilaterals: H at ACA's own scale equal to the oracle's
    tensorised ACA (float64), and the reverse mode to both point sets within
    float rounding of float64 autograd."""
    require_gpu()
    import paper_2402_18008_amd as hgpu
    src, dst, _ = synth.quadruples(B, 40 + B)
    s32, d32 = np.ascontiguousarray(src.T), np.ascontiguousarray(dst.T)
    s, d = torch.from_numpy(s32).cuda(), torch.from_numpy(d32).cuda()
    announce(f"aca general fwd/bwd B={B}")
    H = hgpu.hg_aca_fwd(s, d).cpu().numpy().reshape(B, 3, 3)
    s64, d64 = torch.from_numpy(s32.astype(np.float64)), torch.from_numpy(d32.astype(np.float64))
    Hr = ow.h_aca(s64, d64).numpy()
    assert (np.abs(H - Hr).max(axis=(1, 2)) <= 1e-12 * np.abs(Hr).max(axis=(1, 2))).all()
    rng = np.random.default_rng(B)
    gH = rng.normal(size=(B, 9))
    gs, gd = hgpu.hg_aca_bwd(s, d, torch.from_numpy(gH).cuda())
    gsr, gdr = ow.aca_vjp(s64, d64, torch.from_numpy(gH).reshape(B, 3, 3))
    g = np.concatenate([gs.cpu().numpy(), gd.cpu().numpy()], axis=1)
    gr = np.concatenate([gsr.numpy(), gdr.numpy()], axis=1)
    assert rel(g, gr).max() < 1e-6
    # the same products through ACA's polynomial form (eq. H_11)
    gsp, gdp = ow.aca_poly_vjp(s64, d64, torch.from_numpy(gH).reshape(B, 3, 3))
    assert rel(g, np.concatenate([gsp.numpy(), gdp.numpy()], axis=1)).max() < 1e-6
    # one side only
    _, gd2 = hgpu.hg_aca_bwd(s, d, torch.from_numpy(gH).cuda(), want_src=False)
    torch.cuda.synchronize()
    assert torch.equal(gd2.cpu(), gd.cpu())


def test_general_aca_in_the_photometric_pipeline():
    """With the square's corners as the source quadrilateral, the general solver
    gives the same loss and offset gradient as the rectangle solver (the loss
    does not depend on the scale of H), and both match float64 autograd
    through the DLT solve."""
    require_gpu()
    import paper_2402_18008_amd as hgpu
    pb = synth.patches(16, 23, size=64, sigma=3.0, max_shift=8, max_offset=12.0)
    # offsets on a 2^-10 grid, so corner + offset is exact in float32 as in double
    pb.offsets = (np.round(pb.offsets * 1024.0) / 1024.0).astype(np.float32)
    corners = ow.square_corners(64, torch.float32).numpy()          # TL TR BR BL
    mnpq = [0, 1, 3, 2]                                               # -> M N P Q
    src = torch.from_numpy(np.tile(corners[mnpq].reshape(1, 8), (16, 1))).cuda()
    off = torch.from_numpy(pb.offsets).cuda().requires_grad_(True)
    img = torch.from_numpy(pb.img).cuda()
    tgt = torch.from_numpy(pb.tgt).cuda()
    announce("aca general in the warp-l1 pipeline, 16 patches 64x64")
    dst = (src.reshape(16, 4, 2) + off[:, mnpq]).reshape(16, 8)
    L = hgpu.WarpL1.apply(hgpu.ACAGeneral.apply(src, dst), img, tgt)
    (g,) = torch.autograd.grad(L.sum(), off)
    Lr_, gr_ = run_pipeline(pb)
    L, g = L.detach().cpu().numpy(), g.cpu().numpy()
    assert np.allclose(L, Lr_, rtol=1e-6, atol=0)
    assert rel(g, gr_).max() < 1e-5
    compare_oracle(pb, L, g, slice(None), "general ACA 64x64")


def _refine_case():
    pb = synth.patches(8, 31, size=48, sigma=3.0, max_shift=4, max_offset=6.0)
    rng = np.random.default_rng(0)
    true = np.repeat(-pb.shift[:, None, :].astype(np.float32), 4, axis=1)
    off0 = (true + rng.uniform(-1.5, 1.5, true.shape)).astype(np.float32)
    return pb, off0


def test_refine_against_oracle_and_graph_replays():
    """Six refinement iterations (solve, warp + L1 backward, reverse mode,
    step) against the oracle's loop; the captured graph replays the eager
    result bit for bit, with the offsets reset by eager work between
    replays."""
    require_gpu()
    import paper_2402_18008_amd as hgpu
    pb, off0 = _refine_case()
    img = torch.from_numpy(pb.img).cuda()
    tgt = torch.from_numpy(pb.tgt).cuda()
    off = torch.from_numpy(off0).cuda()
    announce("refine eager B=8 48x48 iters=6")
    R = hgpu.Refine(img, tgt, off, iters=6, step=20.0)
    R.run()
    torch.cuda.synchronize()
    o_gpu, L_gpu = off.cpu().numpy(), R.loss.cpu().numpy()
    o_ref, L_ref = ow.refine_ref(off0, pb.img, pb.tgt, 6, 20.0)
    assert np.abs(o_gpu - o_ref).max() < 1e-4, np.abs(o_gpu - o_ref).max()
    assert np.allclose(L_gpu, L_ref.numpy(), rtol=1e-5, atol=0)
    announce("refine graph replays")
    G = R.graph()
    for _ in range(3):
        off.copy_(torch.from_numpy(off0))
        torch.cuda.synchronize()
        G.launch()
        torch.cuda.synchronize()
        assert np.array_equal(off.cpu().numpy(), o_gpu)
        assert np.array_equal(R.loss.cpu().numpy(), L_gpu)
    G.close()
    # zero iterations: offsets untouched, loss at the start
    off.copy_(torch.from_numpy(off0))
    R0 = hgpu.Refine(img, tgt, off, iters=0, step=20.0)
    R0.run()
    L0 = hgpu.photometric_loss(off, img, tgt)
    torch.cuda.synchronize()
    assert np.array_equal(off.cpu().numpy(), off0)
    assert torch.equal(R0.loss, L0)


def test_fused_pipeline_equals_separate_stages():
    """The recomputing fused launches do the arithmetic of the separate ACA,
    warp and reverse-mode kernels in the same order: the results are
    identical, on square and non-square patches. The single-pass form (its
    own launch shape and sum order; the gradient scaled by grad_loss after
    the pass) agrees within 1e-6 (loss) and 1e-5 (gradient)."""
    require_gpu()
    for B, h, w, seed in ((64, 128, 128, 4), (7, 37, 53, 5)):
        rng = np.random.default_rng(seed)
        img = torch.from_numpy(rng.normal(size=(B, h, w)).astype(np.float32)).cuda()
        tgt = torch.from_numpy(rng.normal(size=(B, h, w)).astype(np.float32)).cuda()
        o = rng.uniform(-8, 8, (B, 4, 2)).astype(np.float32)
        announce(f"fused vs separate B={B} {h}x{w}")
        res = []
        for fused in ("recompute", False, True):
            off = torch.from_numpy(o).cuda().requires_grad_(True)
            import paper_2402_18008_amd as hgpu
            L = hgpu.photometric_loss(off, img, tgt, fused=fused)
            gl = torch.from_numpy(rng.random(B).astype(np.float32)).cuda() if not res else res[0][2]
            (g,) = torch.autograd.grad(L, off, gl)
            torch.cuda.synchronize()
            res.append((L.detach().cpu(), g.cpu(), gl))
        assert torch.equal(res[0][0], res[1][0])
        assert torch.equal(res[0][1], res[1][1])
        assert torch.allclose(res[2][0], res[0][0], rtol=1e-6, atol=0)
        assert rel(res[2][1].numpy(), res[0][1].numpy()).max() < 1e-5
