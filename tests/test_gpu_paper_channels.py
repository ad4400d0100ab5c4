"""The paper's own channel layout (Sec. 3.2, Eq. (1), Fig. 2) as a device
channel mode: double buffers of 2r slots and the delay-token buffer of
3r + 1 slots with the slot 3r -> 0 copy.  Checked on the device against the
Fig. 2 golden trace (which frame sits in which slot), against the oracle's
FIFO order, on the paper's motion-detection pipeline (bit-exact frames,
three actors and fused), and its footprint against Table 1 (3.46 MB)."""
import os

import numpy as np
import pytest

from oracle import fifo_layout as fl
from oracle import md_paper as omd
from oracle.dataflow import Fifo
from workloads import paper_motion

from helpers import say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fig2_delay_token_r4.txt")


def _fig2_ops():
    ops = []
    for line in open(GOLDEN):
        t = line.split("#")[0].split()
        if t and t[0] in ("write", "read"):
            ops.append((t[0], int(t[1]), int(t[2]), (int(t[4]), int(t[5])) if len(t) > 3 else None))
    return ops


def run_paper_layout(frames, batches, fused, threshold=20, rate=4):
    """Push/fire/pop in firing batches of at most two (the double buffers'
    limit), every channel in the paper's layout."""
    from paper_1611_03226_amd.graph import Graph
    n, H, W = frames.shape
    out = np.zeros((sum(batches) * rate, H, W), np.uint8)
    with Graph(0) as G:
        p = G.paper_motion_pipeline(W, H, threshold, rate, layout="paper")
        pos = got = 0
        for b in batches:
            k = b * rate
            G.push(p.inp, frames[pos:pos + k])
            pos += k
            if fused:
                assert p.fire_chain(G, b) == b
            else:
                p.fire_all(G, b)
            got += G.pop(p.out, out[got:got + k])
        assert G.status(p.g_delayed)[:2] == (pos, pos + 1)
        G.sync()
    return out


@pytest.mark.parametrize("fused", [False, True])
def test_pipeline_in_paper_layout_bit_exact(fused):
    say(f"paper-layout pipeline fused={fused}")
    w = paper_motion(seed=41, n_frames=4 * 13, width=320, height=240)
    batches = [1, 2, 1, 1, 2, 2, 1, 2, 1]          # 13 firings: the delay buffer wraps four times
    out = run_paper_layout(w.frames, batches, fused)
    assert np.array_equal(out, omd.paper_motion_direct(w.frames, 20))


def test_delay_buffer_follows_fig2_on_the_device():
    """Gauss writes the delay channel (3r + 1 = 13 slots at r = 4), Thres
    reads it; after every step of the Fig. 2 sequence the device slots hold
    the frames the trace places there (D = the all-zero initial frame, slot
    0 a copy of slot 12 after the third write)."""
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    say("paper-layout delay buffer vs Fig. 2")
    r, H, W = 4, 24, 32
    w = paper_motion(seed=42, n_frames=4 * 9, width=W, height=H)
    g = [omd.gauss5(f) for f in w.frames]
    ops = _fig2_ops()
    with Graph(0) as G:
        p = G.paper_motion_pipeline(W, H, 20, r, layout="paper")
        assert D.df_fifo_bytes(G.g, p.g_delayed) == 13 * W * H
        slot_pos = {0: -1}                          # logical token in each slot (-1: D)
        written = read = 0
        for cycle in range(3):
            for op, lo, hi, copy in ops:
                if op == "write":                   # one Gauss firing: frames written .. written+3
                    G.push(p.inp, w.frames[written:written + r])
                    assert G.fire(p.gauss, 1) == 1
                    for s in range(lo, hi + 1):
                        slot_pos[s] = written + s - lo
                    written += r
                    if copy:
                        slot_pos[copy[1]] = slot_pos[copy[0]]
                else:                               # one Thres + Med firing reads slots lo..hi
                    assert G.fire(p.thres, 1) == 1 and G.fire(p.med, 1) == 1
                    out = np.zeros((r, H, W), np.uint8)
                    assert G.pop(p.out, out) == r
                    read += r
                raw = D.df_debug_read_slots(G.g, p.g_delayed).reshape(13, H, W)
                for s, k in slot_pos.items():
                    want = np.zeros((H, W), np.uint8) if k < 0 else g[k]
                    assert np.array_equal(raw[s], want), (cycle, op, lo, s, k)
        G.sync()


def test_host_traffic_keeps_fifo_order():
    """Host pushes and pops through a delay-layout channel of rate 3 (10
    slots) in uneven amounts: the popped stream is the oracle FIFO's."""
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    say("paper-layout host traffic")
    rng = np.random.default_rng(43)
    init = np.array([-7], np.int32)
    with Graph(0) as G:
        f = D.df_fifo_create_paper(G.g, D.DF_I32, 1, 3, 1, init)
        ref = Fifo("ref", (), np.int32, rate=1, initial=init)
        nxt = 0
        got, want = [], []
        for _ in range(60):
            r_, w_, cap = G.status(f)
            assert cap == 9
            k = int(rng.integers(0, cap - (w_ - r_) + 1))
            v = np.arange(nxt, nxt + k, dtype=np.int32)
            nxt += k
            G.push(f, v)
            for t in v:
                ref.write(np.array([t], np.int32))
            m = int(rng.integers(0, (w_ + k - r_) + 1))
            out = np.zeros(m, np.int32)
            assert G.pop(f, out) == m
            got.extend(out.tolist())
            want.extend(int(ref.read(1)[0]) for _ in range(m))
        G.sync()
    assert got == want and len(got) > 100


def test_footprint_matches_table1():
    """All five channels of the motion network in the paper's layout at
    r = 4, 320x240 tokens: 45 frames = 3.456 MB (Table 1: 3.46 MB)."""
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    say("paper-layout footprint")
    with Graph(0) as G:
        p = G.paper_motion_pipeline(320, 240, 20, 4, layout="paper")
        total = sum(D.df_fifo_bytes(G.g, f) for f in (p.inp, p.g_cur, p.g_delayed, p.thr, p.out))
    want = sum(fl.capacity_bytes(s, r, d) for s, r, d in fl.paper_motion_channels(320, 240, 4))
    assert total == want == 45 * 76800
    assert round(total / 1e6, 2) == 3.46


def test_paper_layout_rejects_other_actors():
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    say("paper-layout connect rules")
    with Graph(0) as G:
        p = D.MotionParams(32, 8, 25, 1, 1)
        a = D.df_actor_create(G.g, D.DF_ACTOR_MOTION, p)
        f = D.df_fifo_create_paper(G.g, D.DF_U8, 256, 4, 0)
        with pytest.raises(D.DFError) as e:
            D.df_connect(G.g, a, D.DF_MD_CUR, f)
        assert e.value.code == D.DF_EINVAL
        with pytest.raises(D.DFError) as e:
            D.df_fifo_create_paper(G.g, D.DF_U8, 256, 4, 2)     # two delay tokens: not in the paper's layout
        assert e.value.code == D.DF_EINVAL
