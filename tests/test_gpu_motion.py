"""GPU parity of the motion actor through the C ABI: emitted masks, frame
indices and token counts bit-exact against the oracle network."""
import numpy as np
import pytest

from oracle import motion as omo
from workloads import motion as gen_motion

from helpers import say

pytestmark = pytest.mark.gpu


def _pow2(n):
    p = 1
    while p < n:
        p <<= 1
    return p


def run_motion_gpu(frames, self_delay=True, batches=None, threshold=25, permille=1):
    from paper_1611_03226_amd.graph import Graph
    n, H, W = frames.shape
    batches = batches or [n]
    with Graph(0) as G:
        ch = G.motion_chain(W, H, threshold, permille, self_delay, cap_in=_pow2(max(batches) + 1),
                            cap_out=_pow2(n))
        pos = 0
        for k in batches:
            G.push(ch.cur, frames[pos:pos + k])
            if not self_delay:
                G.push(ch.prev, frames[pos:pos + k])
            assert G.fire(ch.actor, k) == k
            pos += k
        r, w, _ = G.status(ch.index)
        m = w - r
        masks = np.zeros((m, H, W), np.uint8)
        idx = np.zeros(m, np.int64)
        assert G.pop(ch.mask, masks) == m
        assert G.pop(ch.index, idx) == m
        # every input frame was consumed
        assert G.status(ch.cur)[0] == n
        G.sync()
    return masks, idx


def _check(frames, masks, idx, threshold=25, permille=1):
    ref_m, ref_i = omo.run_motion(frames, threshold, permille)
    assert np.array_equal(idx, ref_i)
    assert masks.shape == ref_m.shape
    assert np.array_equal(masks, ref_m)


@pytest.mark.parametrize("self_delay", [True, False])
def test_ragged_frames_match_oracle(self_delay):
    say(f"motion ragged self_delay={self_delay}")
    w = gen_motion(seed=11, n_frames=24, width=333, height=251, rect_min=12, rect_max=80, segment=5)
    masks, idx = run_motion_gpu(w.frames, self_delay)
    print(f"emitted {len(idx)} of 24")
    _check(w.frames, masks, idx)
    assert len(idx) > 0


def test_batch_splits_and_per_frame_are_identical():
    w = gen_motion(seed=12, n_frames=20, width=200, height=120, rect_min=10, rect_max=50, segment=4)
    ref = None
    for b in ([20], [1] * 20, [7, 6, 7]):
        say(f"motion split {b[:3]}")
        masks, idx = run_motion_gpu(w.frames, True, b)
        if ref is None:
            ref = (masks, idx)
            _check(w.frames, masks, idx)
        assert np.array_equal(idx, ref[1]) and np.array_equal(masks, ref[0])


def test_emission_boundary_and_thresholds():
    say("motion boundary")
    prev = np.zeros((100, 100), np.uint8)
    f1 = prev.copy()
    f1[10:13, 10:13] = 90          # 9 px: no output (needs >= 10 for 100x100)
    f2 = prev.copy()
    f2[10:13, 10:14] = 90          # 12 px: emitted
    def block(v):
        f = f2.copy()
        f[50:60, 50:60] = v
        return f
    # f2 vs f2: nothing; 26 vs 0: changed; 51 vs 26 (diff 25): unchanged;
    # 77 vs 51 (diff 26): changed
    frames = np.stack([prev, f1, prev, f2, f2, block(26), block(51), block(77)])
    for sd in (True, False):
        masks, idx = run_motion_gpu(frames, sd)
        _check(frames, masks, idx)
        assert idx.tolist() == [3, 5, 7]


def test_frame_edges_and_corners():
    """Blocks touching every border and corner; the out-of-frame rules decide."""
    say("motion borders")
    rng = np.random.default_rng(3)
    H, W = 70, 130
    frames = np.zeros((6, H, W), np.uint8)
    for t in range(1, 6):
        f = frames[t - 1].copy()
        for (y, x) in [(0, 0), (0, W - 2), (H - 2, 0), (H - 2, W - 2), (0, 60), (35, 0), (H - 1, 64)]:
            f[y:y + 2, x:x + 2] = rng.integers(60, 256)
        f[30:34, 62:67] = rng.integers(0, 256)
        frames[t] = f
    masks, idx = run_motion_gpu(frames, True, permille=0)
    _check(frames, masks, idx, permille=0)


@pytest.mark.parametrize("self_delay", [True, False])
def test_full_size_workload_bit_exact(self_delay):
    """300 frames of 1920x1080 in one batch; every emitted mask compared."""
    say(f"motion 300x1080p self_delay={self_delay}")
    w = gen_motion()
    masks, idx = run_motion_gpu(w.frames, self_delay)
    counts = omo.frame_counts(w.frames)
    want = [t for t in range(len(counts)) if omo.emits(counts[t], 1920, 1080)]
    assert idx.tolist() == want
    prev = np.zeros_like(w.frames[0])
    k = 0
    for t in range(len(w.frames)):
        if k < len(want) and want[k] == t:
            m, c = omo.detect(w.frames[t], prev)
            assert np.array_equal(masks[k], m), t
            k += 1
        prev = w.frames[t]
    print(f"emitted {len(idx)} of 300")


@pytest.mark.parametrize("self_delay", [True, False])
def test_wide_frames_span_several_column_chunks(self_delay):
    """2100 px rows need two 62-word column chunks; 4100 px three (and a
    partial last word); 9 frames leave a partial frame chunk."""
    for W in (2100, 4100):
        say(f"motion wide W={W} self_delay={self_delay}")
        w = gen_motion(seed=13, n_frames=9, width=W, height=45, rect_min=10, rect_max=40, segment=3)
        masks, idx = run_motion_gpu(w.frames, self_delay, permille=0)
        _check(w.frames, masks, idx, permille=0)


@pytest.mark.parametrize("threshold", [0, 100, 255])
@pytest.mark.parametrize("self_delay", [True, False])
def test_thresholds_match_oracle(threshold, self_delay):
    """Other difference thresholds than 25: 0 (any change counts), 100, and
    255 (nothing can exceed it: no frame emits)."""
    say(f"motion threshold={threshold} self_delay={self_delay}")
    w = gen_motion(seed=14, n_frames=12, width=320, height=97, rect_min=12, rect_max=60, segment=3)
    frames = w.frames.copy()
    # large steps so that a threshold of 100 still finds changed blocks
    frames[5, 20:60, 30:90] = 255
    frames[6, 20:60, 30:90] = 0
    masks, idx = run_motion_gpu(frames, self_delay, threshold=threshold, permille=1)
    _check(frames, masks, idx, threshold=threshold, permille=1)
    if threshold == 255:
        assert len(idx) == 0
    else:
        assert len(idx) > 0
