"""Pins for the oracle's 4-point-offset pipeline (CPU only, torch float64)."""
import numpy as np
import pytest
import torch
from scipy import ndimage

import synth
from oracle import homography as hg
from oracle import warp


@pytest.fixture(scope="module")
def small():
    pb = synth.patches(6, 11, size=32, sigma=2.0, max_shift=4, max_offset=6.0)
    return pb


def test_bilinear_matches_scipy(small):
    img = torch.as_tensor(small.img, dtype=torch.float64)
    rng = np.random.default_rng(0)
    sx = torch.as_tensor(rng.uniform(-3, 35, (6, 500)))
    sy = torch.as_tensor(rng.uniform(-3, 35, (6, 500)))
    got = warp.bilinear_zero(img, sx, sy).numpy()
    for b in range(6):
        ref = ndimage.map_coordinates(small.img[b].astype(np.float64), [sy[b].numpy(), sx[b].numpy()],
                                      order=1, mode="grid-constant", cval=0.0)
        assert np.abs(got[b] - ref).max() < 1e-12


def test_zero_offsets_identity(small):
    img = torch.as_tensor(small.img, dtype=torch.float64)
    H = warp.h_dlt(torch.zeros(6, 4, 2, dtype=torch.float64), 32)
    assert torch.allclose(H, torch.eye(3, dtype=torch.float64).expand(6, 3, 3), atol=1e-12)
    Iw = warp.warp(img, H)
    assert torch.abs(Iw - img).max() < 1e-9


def test_integer_translation_shifts(small):
    img = torch.as_tensor(small.img, dtype=torch.float64)
    off = torch.zeros(6, 4, 2, dtype=torch.float64)
    off[:, :, 0] = 3.0
    off[:, :, 1] = -2.0
    Iw = warp.warp(img, warp.h_dlt(off, 32)).numpy()
    ref = np.zeros_like(small.img, dtype=np.float64)
    # I_w(x, y) = I(x - 3, y + 2)
    ref[:, 0:30, 3:32] = small.img[:, 2:32, 0:29]
    assert np.abs(Iw - ref).max() < 1e-9


def test_rect_solver_matches_dlt():
    rng = np.random.default_rng(1)
    off = torch.as_tensor(rng.uniform(-32, 32, (50, 4, 2)))
    assert hg.herr(warp.h_rect(off, 128).numpy(), warp.h_dlt(off, 128).numpy()).max() < 1e-12


def test_rect_jacobian_finite_differences():
    rng = np.random.default_rng(2)
    off = torch.as_tensor(rng.uniform(-32, 32, (4, 4, 2)), dtype=torch.float64).requires_grad_(True)
    gH = torch.as_tensor(rng.normal(size=(4, 3, 3)))
    (g,) = torch.autograd.grad((warp.h_rect(off, 128) * gH).sum(), off)
    h = 1e-5
    fd = torch.zeros_like(g)
    with torch.no_grad():
        for k in range(4):
            for c in range(2):
                e = torch.zeros_like(off)
                e[:, k, c] = h
                fd[:, k, c] = ((warp.h_rect(off + e, 128) - warp.h_rect(off - e, 128)) * gH).sum((1, 2)) / (2 * h)
    assert torch.allclose(g, fd, rtol=1e-7, atol=1e-6 * g.abs().max().item())


def test_loss_gradient_finite_differences(small):
    off = torch.as_tensor(small.offsets, dtype=torch.float64)
    L, g = warp.loss_and_grad(off, small.img, small.tgt)
    fd = warp.loss_fd_grad(off, small.img, small.tgt, h=1e-6)
    rel = (g - fd).norm(dim=(1, 2)) / g.norm(dim=(1, 2))
    assert rel.max() < 1e-4
    # the solver choice does not change the loss (H only matters up to scale)
    L2, g2 = warp.loss_and_grad(off, small.img, small.tgt, solver=warp.h_rect)
    assert torch.allclose(L, L2, rtol=1e-12)
    assert torch.allclose(g, g2, rtol=1e-8, atol=1e-12)


def test_loss_zero_at_true_shift():
    # the target is the source displaced by an integer shift: offsets equal to
    # minus that shift align them everywhere both are defined
    pb = synth.patches(3, 5, size=32, sigma=2.0, max_shift=3)
    off = np.zeros((3, 4, 2))
    off[:, :, 0] = -pb.shift[:, 0, None]
    off[:, :, 1] = -pb.shift[:, 1, None]
    H = warp.h_dlt(torch.as_tensor(off), 32)
    Iw = warp.warp(torch.as_tensor(pb.img, dtype=torch.float64), H).numpy()
    # in the overlap, I_w equals T up to the independent standardisation of each crop
    for b in range(3):
        sx, sy = pb.shift[b]
        ys = slice(max(0, -sy), 32 - max(0, sy))
        xs = slice(max(0, -sx), 32 - max(0, sx))
        a = Iw[b][ys, xs].ravel()
        t = pb.tgt[b][ys, xs].ravel().astype(np.float64)
        assert np.corrcoef(a, t)[0, 1] > 0.999999


def test_general_aca_matches_dlt_and_finite_differences():
    """The tensorised general ACA is the homography through the four
    correspondences, and its autograd reverse mode agrees with central finite
    differences of the float64 solver."""
    src, dst, _ = synth.quadruples(6, 21)
    s = torch.as_tensor(src.T.astype(np.float64))
    d = torch.as_tensor(dst.T.astype(np.float64))
    H = warp.h_aca(s, d).numpy()
    assert hg.herr(H, hg.dlt64(src.astype(np.float64), dst.astype(np.float64))).max() < 1e-10
    rng = np.random.default_rng(3)
    gH = torch.as_tensor(rng.normal(size=(6, 3, 3)))
    gs, gd = warp.aca_vjp(s, d, gH)
    for x, g, which in ((s, gs, 0), (d, gd, 1)):
        fd = torch.zeros_like(g)
        for k in range(8):
            e = torch.zeros_like(x)
            e[:, k] = 1e-4
            a = (s + e, d) if which == 0 else (s, d + e)
            b = (s - e, d) if which == 0 else (s, d - e)
            fd[:, k] = ((warp.h_aca(*a) - warp.h_aca(*b)) * gH).sum((1, 2)) / 2e-4
        scale = g.abs().max(dim=1, keepdim=True).values
        assert ((g - fd).abs() <= 1e-7 * scale).all(), (which, (g - fd).abs().max())


def test_polynomial_form_has_the_same_derivative():
    """The polynomial form (eq. H_11 with the f3 reading) is the same function
    as the product form at the same scale, so reverse mode through either gives
    the same vector-Jacobian products; central finite differences of the
    polynomial form agree too."""
    src, dst, _ = synth.quadruples(64, 22)
    s = torch.as_tensor(src.T.astype(np.float64))
    d = torch.as_tensor(dst.T.astype(np.float64))
    Hp, Ha = warp.h_aca_poly(s, d), warp.h_aca(s, d)
    scale = Ha.abs().amax(dim=(1, 2), keepdim=True)
    assert ((Hp - Ha).abs() <= 1e-12 * scale).all()
    rng = np.random.default_rng(4)
    gH = torch.as_tensor(rng.normal(size=(64, 3, 3)))
    gps, gpd = warp.aca_poly_vjp(s, d, gH)
    gas, gad = warp.aca_vjp(s, d, gH)
    for gp, ga in ((gps, gas), (gpd, gad)):
        sc = ga.abs().max(dim=1, keepdim=True).values
        assert ((gp - ga).abs() <= 1e-11 * sc).all()
    for k in range(8):
        e = torch.zeros_like(d)
        e[:, k] = 1e-4
        fd = ((warp.h_aca_poly(s, d + e) - warp.h_aca_poly(s, d - e)) * gH).sum((1, 2)) / 2e-4
        assert ((gpd[:, k] - fd).abs() <= 1e-7 * gpd.abs().max(dim=1).values).all()


def test_refinement_moves_towards_the_true_offsets():
    """Gradient-step refinement on patches whose target is an integer
    translation of the source: six steps from a perturbed start reduce every
    patch's loss and its distance to the true offsets (-shift on every
    corner); a step of the wrong sign would increase both. Zero iterations
    return the input."""
    pb = synth.patches(4, 31, size=48, sigma=3.0, max_shift=4, max_offset=6.0)
    rng = np.random.default_rng(0)
    true = np.repeat(-pb.shift[:, None, :].astype(np.float32), 4, axis=1)
    off0 = (true + rng.uniform(-1.5, 1.5, true.shape)).astype(np.float32)
    L0 = warp.loss(torch.as_tensor(off0, dtype=torch.float64),
                   torch.as_tensor(pb.img, dtype=torch.float64),
                   torch.as_tensor(pb.tgt, dtype=torch.float64))
    off, L = warp.refine_ref(off0, pb.img, pb.tgt, 6, 20.0)
    e0 = np.abs(off0 - true).max(axis=(1, 2))
    e6 = np.abs(off - true).max(axis=(1, 2))
    assert (e6 < 0.7 * e0).all(), (e0, e6)
    assert (L < L0).all()
    same, _ = warp.refine_ref(off0, pb.img, pb.tgt, 0, 20.0)
    assert np.array_equal(same, off0)
