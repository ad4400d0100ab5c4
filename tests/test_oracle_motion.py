"""Pins for the motion-detection oracle (CPU only): hand-made frames with
known answers, scipy.ndimage morphology, a pure-Python brute force, the
emission boundary, and the one-frame delay of the initial token (Sec. 4.1)."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import motion
from workloads import motion as gen_motion


def _brute(cur, prev, thr):
    H, W = cur.shape
    m0 = [[abs(int(cur[y, x]) - int(prev[y, x])) > thr for x in range(W)] for y in range(H)]

    def nb(y, x):
        return [(y + dy, x + dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                if 0 <= y + dy < H and 0 <= x + dx < W]
    e = [[all(m0[a][b] for a, b in nb(y, x)) for x in range(W)] for y in range(H)]
    o = [[any(e[a][b] for a, b in nb(y, x)) for x in range(W)] for y in range(H)]
    return np.array(o, bool)


def test_matches_pure_python_brute_force():
    rng = np.random.default_rng(0)
    for H, W in [(1, 1), (2, 3), (5, 7), (9, 4)]:
        cur = rng.integers(0, 256, (H, W)).astype(np.uint8)
        prev = rng.integers(0, 256, (H, W)).astype(np.uint8)
        cur[:, : W // 2] = prev[:, : W // 2]
        mask, count = motion.detect(cur, prev, 25)
        want = _brute(cur, prev, 25)
        assert np.array_equal(mask, want.astype(np.uint8) * 255)
        assert count == want.sum()


def test_matches_scipy_ndimage_opening_with_border_rules():
    rng = np.random.default_rng(1)
    st = np.ones((3, 3), bool)
    for _ in range(20):
        m = rng.random((23, 31)) < rng.uniform(0.3, 0.95)
        e = ndi.binary_erosion(m, structure=st, border_value=1)
        o = ndi.binary_dilation(e, structure=st, border_value=0)
        assert np.array_equal(motion.erode3x3(m), e)
        assert np.array_equal(motion.dilate3x3(motion.erode3x3(m)), o)


def test_threshold_is_strict_at_25():
    prev = np.zeros((8, 8), np.uint8)
    for d, expect in [(25, 0), (26, 9)]:
        cur = prev.copy()
        cur[2:5, 2:5] = d
        _, count = motion.detect(cur, prev, 25)
        assert count == expect
    cur = np.full((8, 8), 100, np.uint8)
    prev2 = np.full((8, 8), 126, np.uint8)       # |100-126| = 26 over the whole frame
    assert motion.detect(cur, prev2, 25)[1] == 64


def test_isolated_pixel_removed_block_kept_border_block_kept():
    prev = np.zeros((10, 12), np.uint8)
    cur = prev.copy()
    cur[1, 1] = 200                              # isolated: erased by erosion
    cur[5:8, 6:9] = 200                          # 3x3 block survives unchanged
    mask, count = motion.detect(cur, prev, 25)
    assert count == 9 and mask[5:8, 6:9].all() and mask.sum() == 9 * 255
    cur2 = prev.copy()
    cur2[0:2, 0:2] = 200                         # 2x2 in the corner: out-of-frame counts as set
    mask2, count2 = motion.detect(cur2, prev, 25)
    assert count2 == 4 and mask2[0:2, 0:2].all()
    cur3 = prev.copy()
    cur3[4:6, 4:6] = 200                         # 2x2 inside: removed
    assert motion.detect(cur3, prev, 25)[1] == 0


def test_emission_boundary():
    W, H = 1920, 1080                            # 0.1 % of 2,073,600 px = 2073.6
    assert not motion.emits(2073, W, H, 1)
    assert motion.emits(2074, W, H, 1)
    # small frame: 100x100 -> needs count >= 10
    prev = np.zeros((100, 100), np.uint8)
    f1 = prev.copy()
    f1[10:13, 10:13] = 90                       # 9 px: no output
    f2 = prev.copy()
    f2[10:13, 10:14] = 90                       # 12 px: emits
    frames = np.stack([prev, f1, prev, f2])
    masks, idx = motion.run_motion(frames)
    # frame 0 vs zero initial token: identical -> none; f1 vs 0: 9 -> none;
    # prev vs f1: 9 -> none; f2 vs prev: 12 -> emit
    assert idx.tolist() == [3]
    assert masks.shape == (1, 100, 100) and (masks[0] > 0).sum() == 12


def test_initial_token_is_a_zero_frame_and_identical_frames_emit_nothing():
    rng = np.random.default_rng(2)
    f = rng.integers(0, 256, (40, 50)).astype(np.uint8)
    masks, idx = motion.run_motion(np.stack([f, f, f]))
    assert idx.tolist() == [0]                   # frame 0 is diffed against black
    want, _ = motion.detect(f, np.zeros_like(f), 25)
    assert np.array_equal(masks[0], want)


def test_network_agrees_with_counts_and_schedules():
    w = gen_motion(seed=7, n_frames=12, width=160, height=96, rect_min=8, rect_max=40, segment=4)
    masks, idx = motion.run_motion(w.frames)
    counts = motion.frame_counts(w.frames)
    emit = [t for t in range(12) if motion.emits(counts[t], 160, 96)]
    assert idx.tolist() == emit
    for k, t in enumerate(emit):
        prev = w.frames[t - 1] if t else np.zeros_like(w.frames[0])
        assert np.array_equal(masks[k], motion.detect(w.frames[t], prev)[0])
    for seed in (1, 2):
        m2, i2 = motion.MotionNetwork(w.frames).run("random", seed)
        assert np.array_equal(m2, masks) and np.array_equal(i2, idx)
