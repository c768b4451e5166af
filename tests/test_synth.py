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
