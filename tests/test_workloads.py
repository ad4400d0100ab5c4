"""Seeded generators: reproducible, and with the stated distributions."""
import numpy as np

from workloads import (adaptation, dpd_chain, dpd_instances, dpd_scale, motion,
                       ofdm_like, papr_db)


def test_seeds_reproduce():
    a, b = dpd_chain(), dpd_chain()
    assert np.array_equal(a.x, b.x) and np.array_equal(a.ctrl, b.ctrl) and np.array_equal(a.h, b.h)
    m1 = motion(seed=9, n_frames=3, width=64, height=48, rect_min=8, rect_max=16)
    m2 = motion(seed=9, n_frames=3, width=64, height=48, rect_min=8, rect_max=16)
    assert np.array_equal(m1.frames, m2.frames)
    c = dpd_chain(seed=2)
    assert not np.array_equal(a.x, c.x)


def test_chain_shapes_and_ranges():
    w = dpd_chain()
    assert w.x.shape == (16384,) and w.x.dtype == np.complex64
    assert w.ctrl.min() >= 1 and w.ctrl.max() <= 5 and len(w.ctrl) == 64
    assert w.h.shape == (5, 8) and w.h[0, 0] == 1
    assert abs(np.sqrt(np.mean(np.abs(w.x) ** 2)) - 1.0) < 0.02


def test_ofdm_like_band_limit_and_papr():
    rng = np.random.default_rng(0)
    x = ofdm_like(rng, 1 << 16)
    spec = np.abs(np.fft.fft(x.astype(np.complex128))) ** 2
    f = np.abs(np.fft.fftfreq(len(x)))
    out_band = spec[f > 0.42].sum() / spec.sum()
    assert out_band < 0.01                          # clipping regrowth only
    assert 8.5 < papr_db(x) <= 10.01
    assert abs(np.mean(np.abs(x) ** 2) - 1.0) < 1e-5


def test_scale_small_instance_properties():
    w = dpd_scale(n_samples=1 << 16, r=4096)
    assert w.n_firings == 16 and w.ctrl.min() >= 1 and w.ctrl.max() <= 10
    scale = np.abs(w.h[1:, :]).mean(axis=1)
    assert scale[-1] < scale[0]                     # factorial scaling of high orders


def test_instances_lengths():
    w = dpd_instances(with_signals=False)
    assert len(w.lengths) == 1024
    assert (w.lengths % 1024 == 0).all()
    assert w.lengths.min() >= 1024 and w.lengths.max() <= 262144
    assert 15e6 < w.lengths.sum() < 40e6
    assert w.n_branches.min() >= 1 and w.n_branches.max() <= 10


def test_adaptation_workload():
    w = adaptation(n_streams=2, length=1024)
    assert w.x.shape == (2, 1024)
    assert abs(np.sqrt(np.mean(np.abs(w.x) ** 2)) - 0.25) < 0.02
    assert w.a.shape == (4, 4) and w.a[0, 0] == 1 and w.h0[0, 0] == 1


def test_paper_motion_frames():
    from workloads import paper_motion
    a, b = paper_motion(seed=4, n_frames=5), paper_motion(seed=4, n_frames=5)
    assert a.frames.shape == (5, 240, 320) and a.frames.dtype == np.uint8
    assert np.array_equal(a.frames, b.frames)
    assert a.width * a.height == 76800                  # the paper's 76,800-byte tokens
    # consecutive frames differ (noise and moving rectangles), but mostly by little
    d = np.abs(a.frames[1].astype(int) - a.frames[0].astype(int))
    assert 0 < np.median(d) <= 8
