"""Pins for the oracle of the paper's motion-detection pipeline (Sec. 4.1),
CPU only: the binomial weights from Pascal's triangle, closed-form impulse
and linear-ramp responses of the Gaussian, scipy.ndimage filters with
replicated borders, pure-Python brute force of Thres and Med, and the
network (rate 4, one initial token) against the per-frame composition."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import md_paper as md


def test_gauss_weights_are_binomial():
    w = np.array([[math.comb(4, i) * math.comb(4, j) for j in range(5)] for i in range(5)])
    assert np.array_equal(md.GAUSS_KERNEL, w)
    assert md.GAUSS_KERNEL.sum() == 256


def test_gauss_impulse_closed_form():
    # impulse of 255 in a zero frame: response (255*w + 128) >> 8 at each offset
    f = np.zeros((11, 11), np.uint8)
    f[5, 5] = 255
    g = md.gauss5(f)
    want = {36: 36, 24: 24, 16: 16, 6: 6, 4: 4, 1: 1}   # (255 w + 128) >> 8 == w for these w
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            w = math.comb(4, dy + 2) * math.comb(4, dx + 2)
            assert g[5 + dy, 5 + dx] == want[w] == (255 * w + 128) >> 8
    g[3:8, 3:8] = 0
    assert not g.any()


def test_gauss_preserves_linear_ramps_away_from_column_edges():
    # the kernel is symmetric with weights summing to 256: a linear image is a
    # fixed point wherever no neighbour column is clamped
    H, W = 12, 20
    y, x = np.mgrid[0:H, 0:W]
    for a, b, c in [(3, 7, 5), (11, 2, 0), (0, 9, 30)]:
        f = (a * x + b * y + c).astype(np.uint8)
        assert f.max() < 256
        g = md.gauss5(f)
        assert np.array_equal(g[:, 2:W - 2], f[:, 2:W - 2])


def test_gauss_matches_scipy_correlate_nearest():
    rng = np.random.default_rng(3)
    for H, W in [(5, 5), (9, 13), (24, 32), (17, 3), (6, 1)]:
        f = rng.integers(0, 256, (H, W)).astype(np.uint8)
        s = ndi.correlate(f.astype(np.int64), md.GAUSS_KERNEL, mode="nearest")
        want = ((s + 128) >> 8).astype(np.uint8)
        want[:2] = f[:2]
        want[H - 2:] = f[H - 2:]
        assert np.array_equal(md.gauss5(f), want)


@pytest.mark.parametrize("H", [1, 2, 3, 4])
def test_gauss_short_frames_are_copied(H):
    f = np.random.default_rng(H).integers(0, 256, (H, 7)).astype(np.uint8)
    assert np.array_equal(md.gauss5(f), f)


def test_gauss_skips_exactly_two_rows_each_side():
    f = np.zeros((8, 6), np.uint8)
    f[::2] = 200                      # stripes: filtering changes every filtered row
    g = md.gauss5(f)
    assert np.array_equal(g[[0, 1, 6, 7]], f[[0, 1, 6, 7]])
    assert (g[2:6] != f[2:6]).all()


def test_thres_brute_force_and_strictness():
    rng = np.random.default_rng(4)
    a = rng.integers(0, 256, (7, 9)).astype(np.uint8)
    b = rng.integers(0, 256, (7, 9)).astype(np.uint8)
    b[0, :] = np.clip(a[0, :].astype(int) + 20, 0, 255)       # |d| == 20 somewhere
    for T in (0, 20, 128, 255):
        t = md.thres(a, b, T)
        for y in range(7):
            for x in range(9):
                d = abs(int(a[y, x]) - int(b[y, x]))
                assert t[y, x] == (255 if d > T else 0)
    assert not md.thres(a, a, 0).any()


def _med_brute(f):
    H, W = f.shape
    out = np.zeros_like(f)
    for y in range(H):
        for x in range(W):
            vals = []
            for dy, dx in ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)):
                yy = min(max(y + dy, 0), H - 1)
                xx = min(max(x + dx, 0), W - 1)
                vals.append(int(f[yy, xx]))
            out[y, x] = sorted(vals)[2]
    return out


def test_med_brute_force_and_scipy():
    rng = np.random.default_rng(5)
    plus = np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]], bool)
    for H, W in [(1, 1), (1, 6), (5, 1), (4, 4), (9, 13)]:
        f = rng.integers(0, 256, (H, W)).astype(np.uint8)
        m = md.med5(f)
        assert np.array_equal(m, _med_brute(f))
        assert np.array_equal(m, ndi.median_filter(f, footprint=plus, mode="nearest"))


def test_med_of_binary_is_majority():
    rng = np.random.default_rng(6)
    f = (rng.random((10, 12)) < 0.5).astype(np.uint8) * 255
    p = np.pad(f.astype(int) // 255, 1, mode="edge")
    votes = p[1:-1, 1:-1] + p[:-2, 1:-1] + p[2:, 1:-1] + p[1:-1, :-2] + p[1:-1, 2:]
    assert np.array_equal(md.med5(f), np.where(votes >= 3, 255, 0).astype(np.uint8))


@pytest.mark.parametrize("policy,seed", [("round_robin", 0), ("random", 1), ("random", 2)])
def test_network_equals_per_frame_composition(policy, seed):
    rng = np.random.default_rng(7)
    frames = rng.integers(0, 256, (10, 9, 11)).astype(np.uint8)
    out = md.run_paper_motion(frames, threshold=20, rate=4, policy=policy, seed=seed)
    assert out.shape == (8, 9, 11)            # two whole rate-4 firings
    direct = md.paper_motion_direct(frames, threshold=20)
    assert np.array_equal(out, direct[:8])


def test_initial_token_is_a_one_frame_delay():
    rng = np.random.default_rng(8)
    frames = rng.integers(0, 256, (8, 6, 7)).astype(np.uint8)
    out = md.run_paper_motion(frames, threshold=10, rate=4)
    zero = np.zeros((6, 7), np.uint8)
    assert np.array_equal(out[0], md.med5(md.thres(md.gauss5(frames[0]), zero, 10)))
    for k in range(1, 8):
        want = md.med5(md.thres(md.gauss5(frames[k]), md.gauss5(frames[k - 1]), 10))
        assert np.array_equal(out[k], want)
    # rate 1 gives the same stream
    assert np.array_equal(md.run_paper_motion(frames, threshold=10, rate=1), out)


def test_static_scene_gives_empty_mask_after_first_frame():
    f = np.random.default_rng(9).integers(0, 256, (8, 10)).astype(np.uint8)
    out = md.paper_motion_direct(np.stack([f] * 5), threshold=5)
    assert not out[1:].any()


def test_eq1_capacity_reproduces_table1_motion_detection():
    # Table 1: the proposed framework's heterogeneous motion detection
    # (320x240 frames, token rate 4 on the GPU) allocates 3.46 MB of channel
    # memory; Eq. (1) over its five channels gives 4*(2*4) + (3*4+1) = 45
    # frames of 76,800 bytes
    from oracle import fifo_layout as fl
    assert fl.capacity_tokens(4, True) == 13 and fl.capacity_tokens(4, False) == 8
    b = fl.network_bytes(fl.paper_motion_channels(320, 240, 4))
    assert b == 45 * 76800
    assert round(b / 1e6, 2) == 3.46


def test_golden_digest_file_is_consistent():
    """The stored full-size digests start where the oracle's first block
    ends up (the first 64 frames recomputed here from the oracle)."""
    import hashlib
    import os
    from workloads import paper_motion
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "md_paper_4096_digests.txt")
    rows = [l.split() for l in open(path) if not l.startswith("#")]
    assert len(rows) == 64 and [int(k) for k, _ in rows] == list(range(0, 4096, 64))
    w = paper_motion(seed=28, n_frames=4096)
    out = md.paper_motion_direct(w.frames[:64], 20)
    assert hashlib.sha256(out.tobytes()).hexdigest() == rows[0][1]
