"""GPU parity of the paper's motion-detection pipeline (Sec. 4.1) through the
C ABI: Gauss, Thres and Med as three static actors joined by device FIFO
channels (one holding the one-frame delay), every output frame bit-exact
against the oracle, on the word path (width a multiple of 4) and the byte
path, across ring wrap-around, batches of uneven size and partial admission."""
import hashlib
import os

import numpy as np
import pytest

from oracle import md_paper as omd
from workloads import paper_motion

from helpers import say

pytestmark = pytest.mark.gpu


def _pow2(n):
    p = 1
    while p < n:
        p <<= 1
    return p


def run_pipeline(frames, threshold=20, rate=4, batches=None, cap=0):
    """Push all frames, fire Gauss/Thres/Med in the given firing batches
    (default: all whole firings at once), pop every output frame."""
    from paper_1611_03226_amd.graph import Graph
    n, H, W = frames.shape
    nf = n // rate
    batches = batches or [nf]
    assert sum(batches) == nf
    cap = cap or _pow2(n + 1)
    out = np.zeros((nf * rate, H, W), np.uint8)
    with Graph(0) as G:
        p = G.paper_motion_pipeline(W, H, threshold, rate, cap=cap)
        pos = got = 0
        for b in batches:
            k = b * rate
            G.push(p.inp, frames[pos:pos + k])
            pos += k
            p.fire_all(G, b)
            got += G.pop(p.out, out[got:got + k])
        assert got == nf * rate
        # token conservation: every channel was read as often as written
        for f in (p.inp, p.g_cur, p.thr, p.out):
            r, w, _ = G.status(f)
            assert r == w == nf * rate
        r, w, _ = G.status(p.g_delayed)
        assert (r, w) == (nf * rate, nf * rate + 1)      # the initial token stays one ahead
        G.sync()
    return out


def _expect(frames, threshold=20):
    return omd.paper_motion_direct(frames, threshold)


def test_paper_size_matches_oracle():
    say("md_paper 320x240 rate 4, 24 frames in batches 2,1,3")
    w = paper_motion(seed=21, n_frames=24)
    out = run_pipeline(w.frames, batches=[2, 1, 3])
    assert np.array_equal(out, _expect(w.frames))


@pytest.mark.parametrize("W,H", [(4, 9), (8, 5), (36, 23), (320, 50), (37, 23), (13, 7), (1, 1), (7, 4),
                                 (16, 3), (5, 17)])
def test_ragged_sizes(W, H):
    say(f"md_paper ragged {W}x{H}")
    rng = np.random.default_rng(W * 1000 + H)
    frames = rng.integers(0, 256, (12, H, W)).astype(np.uint8)
    frames[1::2] = np.clip(frames[0::2].astype(int) + rng.integers(-30, 31, (6, H, W)), 0, 255)
    out = run_pipeline(frames, threshold=12, rate=4, batches=[1, 2])
    assert np.array_equal(out, _expect(frames, 12))


def test_ring_wrap_with_small_capacity():
    say("md_paper ring wrap: capacity 8 frames, 10 firings of rate 4 one at a time")
    w = paper_motion(seed=22, n_frames=40, width=64, height=48)
    out = run_pipeline(w.frames, batches=[1] * 10, cap=8)
    assert np.array_equal(out, _expect(w.frames))


@pytest.mark.parametrize("threshold", [0, 255])
def test_threshold_extremes(threshold):
    say(f"md_paper threshold {threshold}")
    w = paper_motion(seed=23, n_frames=8, width=96, height=40)
    out = run_pipeline(w.frames, threshold=threshold)
    exp = _expect(w.frames, threshold)
    assert np.array_equal(out, exp)
    if threshold == 255:
        assert not out.any()


def test_rate_one_equals_rate_four():
    say("md_paper rate 1 vs rate 4")
    w = paper_motion(seed=24, n_frames=12, width=64, height=32)
    a = run_pipeline(w.frames, rate=1, batches=[5, 7])
    b = run_pipeline(w.frames, rate=4, batches=[3])
    assert np.array_equal(a, b)


def test_single_actors_against_oracle():
    """Each body alone, fed and drained by the host."""
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    rng = np.random.default_rng(25)
    for W, H in [(320, 240), (30, 11)]:
        say(f"md_paper single actors {W}x{H}")
        a = rng.integers(0, 256, (8, H, W)).astype(np.uint8)
        b = rng.integers(0, 256, (8, H, W)).astype(np.uint8)
        with Graph(0) as G:
            p = D.FrameParams(W, H, 4, 40)
            wh = W * H
            ga = D.df_actor_create(G.g, D.DF_ACTOR_GAUSS5, p)
            ta = D.df_actor_create(G.g, D.DF_ACTOR_THRES, p)
            ma = D.df_actor_create(G.g, D.DF_ACTOR_MED5, p)
            f = [G.fifo(D.DF_U8, wh, 16) for _ in range(7)]
            D.df_connect(G.g, ga, D.DF_GAUSS_IN, f[0])
            D.df_connect(G.g, ga, D.DF_GAUSS_OUT, f[1])      # second output left unconnected
            D.df_connect(G.g, ta, D.DF_THRES_CUR, f[2])
            D.df_connect(G.g, ta, D.DF_THRES_PREV, f[3])
            D.df_connect(G.g, ta, D.DF_THRES_OUT, f[4])
            D.df_connect(G.g, ma, D.DF_MED_IN, f[5])
            D.df_connect(G.g, ma, D.DF_MED_OUT, f[6])
            G.push(f[0], a)
            G.push(f[2], a)
            G.push(f[3], b)
            G.push(f[5], a)
            for act in (ga, ta, ma):
                assert G.fire(act, 2) == 2
            g = np.zeros_like(a)
            t = np.zeros_like(a)
            m = np.zeros_like(a)
            assert G.pop(f[1], g) == 8 and G.pop(f[4], t) == 8 and G.pop(f[6], m) == 8
            G.sync()
        for k in range(8):
            assert np.array_equal(g[k], omd.gauss5(a[k]))
            assert np.array_equal(t[k], omd.thres(a[k], b[k], 40))
            assert np.array_equal(m[k], omd.med5(a[k]))


def test_admission_is_all_or_nothing():
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    say("md_paper admission")
    w = paper_motion(seed=26, n_frames=10, width=32, height=16)
    with Graph(0) as G:
        p = G.paper_motion_pipeline(32, 16, 20, 4, cap=16)
        G.push(p.inp, w.frames)                  # 10 frames: two whole firings
        with pytest.raises(D.DFError) as e:
            G.fire(p.gauss, 3)
        assert e.value.code == D.DF_EAGAIN
        assert G.status(p.inp)[:2] == (0, 10)    # nothing changed
        assert G.fire(p.gauss, 3, partial=True) == 2
        assert G.fire(p.thres, 2) == 2
        # Med's output channel holds 16 frames; a third firing's input is missing
        assert G.fire(p.med, 5, partial=True) == 2
        out = np.zeros((8, 16, 32), np.uint8)
        assert G.pop(p.out, out) == 8
        G.sync()
    assert np.array_equal(out, _expect(w.frames[:8]))


def test_profile_per_actor():
    say("md_paper per-actor profile")
    from paper_1611_03226_amd.graph import Graph
    w = paper_motion(seed=27, n_frames=16, width=64, height=32)
    with Graph(0) as G:
        p = G.paper_motion_pipeline(64, 32, 20, 4, cap=32)
        G.profile(True)
        G.push(p.inp, w.frames)
        p.fire_all(G, 4)
        ms_g, n_g = G.profile_read(p.gauss)
        ms_all, n_all = G.profile_read()
        assert n_g == 1 and ms_g > 0
        assert n_all == 2 and ms_all > 0          # Thres and Med still pending
        G.profile(False)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "md_paper_4096_digests.txt")


def check_all_frames_against_oracle_digests(frames, out):
    """Every output frame of the seed-28 4096-frame workload against the
    oracle's block digests (tests/golden, written from the oracle alone); a
    differing block is recomputed by the oracle to name its first bad frame."""
    want = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if not line.startswith("#"):
                k, d = line.split()
                want[int(k)] = d
    assert len(want) == len(out) // 64
    for k0, d in sorted(want.items()):
        if hashlib.sha256(out[k0:k0 + 64].tobytes()).hexdigest() == d:
            continue
        prev = omd.gauss5(frames[k0 - 1]) if k0 else np.zeros(frames.shape[1:], np.uint8)
        for k in range(k0, k0 + 64):
            ref = omd.med5(omd.thres(omd.gauss5(frames[k]), prev, 20))
            assert np.array_equal(out[k], ref), f"frame {k} differs from the oracle"
            prev = omd.gauss5(frames[k])
        raise AssertionError(f"block {k0} differs from its digest but not frame by frame")


def test_full_size_all_frames():
    """4096 frames of 320x240 in one batch of 1024 firings (the bench's
    launch configuration); every output frame against the oracle."""
    say("md_paper 4096 frames 320x240, one batch")
    w = paper_motion(seed=28, n_frames=4096)
    out = run_pipeline(w.frames)
    check_all_frames_against_oracle_digests(w.frames, out)


# ------------------------------------------------------------------ df_fire_pipeline

def run_chain(frames, threshold=20, rate=4, batches=None, cap=0, fused=True):
    """Like run_pipeline, but each batch is one df_fire_pipeline call."""
    from paper_1611_03226_amd.graph import Graph
    n, H, W = frames.shape
    nf = n // rate
    batches = batches or [nf]
    cap = cap or _pow2(n + 1)
    out = np.zeros((nf * rate, H, W), np.uint8)
    with Graph(0) as G:
        p = G.paper_motion_pipeline(W, H, threshold, rate, cap=cap)
        pos = got = 0
        for b in batches:
            k = b * rate
            G.push(p.inp, frames[pos:pos + k])
            pos += k
            assert p.fire_chain(G, b, fused=fused) == b
            got += G.pop(p.out, out[got:got + k])
        assert got == nf * rate
        for f in (p.inp, p.g_cur, p.thr, p.out):
            r, w, _ = G.status(f)
            assert r == w == nf * rate
        assert G.status(p.g_delayed)[:2] == (nf * rate, nf * rate + 1)
        G.sync()
    return out


@pytest.mark.parametrize("fused", [True, False])
def test_chain_paper_size(fused):
    say(f"md_paper chain 320x240 fused={fused}, batches 2,1,3")
    w = paper_motion(seed=31, n_frames=24)
    out = run_chain(w.frames, batches=[2, 1, 3], fused=fused)
    assert np.array_equal(out, _expect(w.frames))


@pytest.mark.parametrize("W,H", [(4, 9), (8, 5), (36, 23), (320, 50), (16, 3), (4, 1), (12, 2), (64, 17),
                                 (37, 23), (13, 7)])
def test_chain_ragged_sizes(W, H):
    say(f"md_paper chain ragged {W}x{H}")
    rng = np.random.default_rng(W * 1000 + H + 7)
    frames = rng.integers(0, 256, (20, H, W)).astype(np.uint8)
    frames[1::2] = np.clip(frames[0::2].astype(int) + rng.integers(-30, 31, (10, H, W)), 0, 255)
    out = run_chain(frames, threshold=12, rate=4, batches=[1, 3, 1])
    assert np.array_equal(out, _expect(frames, 12))


def test_chain_many_frames_per_wave_range_and_ring_wrap():
    # 27 firings of rate 1 in batches that cross the 8-frame ranges of the
    # fused kernel and wrap a 16-frame ring
    say("md_paper chain rate 1, 27 frames, capacity 16")
    w = paper_motion(seed=32, n_frames=27, width=96, height=40)
    out = run_chain(w.frames, rate=1, batches=[9, 1, 12, 5], cap=16)
    assert np.array_equal(out, _expect(w.frames))


def test_chain_falls_back_when_inner_channel_holds_tokens():
    from paper_1611_03226_amd.graph import Graph
    say("md_paper chain after a lone Gauss firing (separate fallback)")
    w = paper_motion(seed=33, n_frames=16, width=64, height=32)
    out = np.zeros((16, 32, 64), np.uint8)
    with Graph(0) as G:
        p = G.paper_motion_pipeline(64, 32, 20, 4, cap=32)
        G.push(p.inp, w.frames)
        assert G.fire(p.gauss, 1) == 1                 # Gauss->Thres now holds 4 frames
        assert p.fire_chain(G, 3) == 3                 # cannot fuse: runs the three actors
        assert G.fire(p.thres, 1) == 1 and G.fire(p.med, 1) == 1
        assert G.pop(p.out, out) == 16
        G.sync()
    assert np.array_equal(out, _expect(w.frames))


def test_chain_admission():
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    say("md_paper chain admission")
    w = paper_motion(seed=34, n_frames=10, width=32, height=16)
    with Graph(0) as G:
        p = G.paper_motion_pipeline(32, 16, 20, 4, cap=16)
        G.push(p.inp, w.frames)
        with pytest.raises(D.DFError) as e:
            p.fire_chain(G, 3)
        assert e.value.code == D.DF_EAGAIN
        assert G.status(p.inp)[:2] == (0, 10)
        assert p.fire_chain(G, 3, partial=True) == 2
        out = np.zeros((8, 16, 32), np.uint8)
        assert G.pop(p.out, out) == 8
        G.sync()
    assert np.array_equal(out, _expect(w.frames[:8]))
    with Graph(0) as G:
        p = G.paper_motion_pipeline(32, 16, 20, 4, cap=16)
        with pytest.raises(D.DFError) as e:
            D.df_fire_pipeline(G.g, p.thres, p.gauss, p.med, 1)
        assert e.value.code == D.DF_EINVAL


def test_chain_full_size_all_frames():
    """4096 frames of 320x240 in one fused batch (the bench's launch); every
    output frame against the oracle (block digests)."""
    say("md_paper chain 4096 frames 320x240, one fused batch")
    w = paper_motion(seed=28, n_frames=4096)
    out = run_chain(w.frames)
    check_all_frames_against_oracle_digests(w.frames, out)


def test_chain_with_host_fed_previous_frames():
    """Gauss's second output unconnected, Thres's previous frames pushed by
    the host: the chain runs as three actors, and its admission counts the
    host-fed channel (no partial chain on DF_EAGAIN)."""
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    say("md_paper chain with host-fed previous frames")
    rng = np.random.default_rng(35)
    W, H = 32, 12
    a = rng.integers(0, 256, (8, H, W)).astype(np.uint8)
    b = rng.integers(0, 256, (8, H, W)).astype(np.uint8)
    with Graph(0) as G:
        p = G.paper_motion_pipeline(W, H, 30, 4, cap=16, second_output=False)
        G.push(p.inp, a)
        G.push(p.g_delayed, b[:3])                  # the channel's zero token + 3 frames: one firing
        with pytest.raises(D.DFError) as e:
            p.fire_chain(G, 2)
        assert e.value.code == D.DF_EAGAIN
        assert G.status(p.inp)[:2] == (0, 8) and G.status(p.g_cur)[:2] == (0, 0)
        assert p.fire_chain(G, 2, partial=True) == 1
        out = np.zeros((4, H, W), np.uint8)
        assert G.pop(p.out, out) == 4
        G.sync()
    prev = np.concatenate([np.zeros((1, H, W), np.uint8), b[:3]])
    for k in range(4):
        assert np.array_equal(out[k], omd.med5(omd.thres(omd.gauss5(a[k]), prev[k], 30)))
