"""Bit-mask control tokens on the fast path (Sec. 4.2: the configuration
selects which set of FIR filters takes part; Sec. 3.1 leaves the token to
rate mapping open): the predistortion actor with control_mode = mask fired
through df_fire and df_fire_many (persistent and graph), against the oracle
network with mask tokens, per-firing rel-RMS, tables bit-exact."""
import numpy as np
import pytest

from oracle import dpd as odpd
from workloads import complex_gaussian, dpd_coeffs, dpd_random

from helpers import DPD_TOL, rel_rms_per_firing, say

pytestmark = pytest.mark.gpu


def _pow2(n):
    p = 1
    while p < n:
        p <<= 1
    return p


def _masks(rng, n, B, p_zero=0.1):
    m = rng.integers(1, 1 << B, n)
    m[rng.random(n) < p_zero] = 0
    return m.astype(np.int32)


def run_mask_chain(G, w, masks, hist="branch", batches=None, cap_x=0):
    n = len(masks)
    batches = batches or [n]
    cap_x = cap_x or _pow2(n * w.r + w.n_delay)
    ch = G.dpd_chain(w.h, w.r, w.n_delay, history=hist, cap_x=cap_x, cap_ctrl=_pow2(n),
                     cap_y=max(cap_x, _pow2(max(batches) * w.r)), control="mask")
    out, pos, xpos = [], 0, 0
    for k in batches:
        need = (pos + k) * w.r - w.n_delay
        if need > xpos:
            G.push(ch.x, np.ascontiguousarray(w.x[xpos:need]))
            xpos = need
        G.push(ch.ctrl, masks[pos:pos + k])
        assert G.fire(ch.actor, k) == k
        buf = np.zeros(k * w.r, np.complex64)
        assert G.pop(ch.y, buf) == k * w.r
        out.append(buf)
        pos += k
    return np.concatenate(out), ch


CASES = [
    # seed, n, r, B_max, M, d, hist, batches, cap_x
    (101, 40, 64, 5, 8, 2, "branch", [13, 27], 2048),
    (102, 36, 300, 10, 16, 0, "branch", [36], 0),
    (103, 30, 257, 10, 16, 3, "shared", [7, 23], 8192),
    (104, 24, 100, 13, 16, 1, "branch", [24], 0),
    (105, 32, 96, 16, 8, 0, "branch", [10, 22], 4096),
    (106, 20, 50, 16, 4, 2, "shared", [1] * 20, 64),
    (107, 18, 20, 6, 5, 1, "branch", [18], 0),          # generic kernel (M = 5)
    (108, 9000, 16, 7, 8, 0, "branch", [9000], 0),      # scan over several passes
]


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}" for c in CASES])
def test_mask_tokens_match_oracle(case):
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    seed, n, r, B, M, d, hist, batches, cap = case
    say(f"dpd mask case {case[:7]}")
    rng = np.random.default_rng(seed)
    w = dpd_random(seed, n_firings=n, r=r, n_branches_max=B, n_taps=M, n_delay=d)
    masks = _masks(rng, n, B)
    with Graph(0) as G:
        y, ch = run_mask_chain(G, w, masks, hist, batches, cap)
        if len(batches) == 1:
            rates, offs, prev = D.df_debug_last_batch(G.g, ch.actor, B, n)
            r_ref, o_ref, p_ref, _ = odpd.firing_tables(masks, B, r, hist, control="mask")
            assert np.array_equal(rates, r_ref)
            assert np.array_equal(offs, o_ref)
            assert np.array_equal(prev, p_ref)
        G.sync()
    ref = odpd.run_dpd(w.x, masks, w.h, r, d, hist=hist, control="mask")
    worst, glob, bad0 = rel_rms_per_firing(y, ref, r)
    print(f"mask case {seed}: worst {worst:.3e} global {glob:.3e}")
    assert worst <= DPD_TOL and bad0 == 0


def test_prefix_masks_equal_count_tokens_bit_for_bit():
    from paper_1611_03226_amd.graph import Graph
    from helpers import run_dpd_chain
    say("dpd prefix masks == counts")
    w = dpd_random(110, n_firings=48, r=128, n_branches_max=10, n_taps=16, n_delay=1)
    masks = ((1 << w.ctrl.astype(np.int64)) - 1).astype(np.int32)
    with Graph(0) as G:
        y_count, _ = run_dpd_chain(G, w)
    with Graph(0) as G:
        y_mask, _ = run_mask_chain(G, w, masks)
    assert np.array_equal(y_count.view(np.float32), y_mask.view(np.float32))


def test_mask_splits_and_per_firing_bit_identical():
    from paper_1611_03226_amd.graph import Graph
    w = dpd_random(111, n_firings=40, r=256, n_branches_max=10, n_taps=16, n_delay=2)
    masks = _masks(np.random.default_rng(111), 40, 10)
    outs = []
    for batches in ([40], [1] * 40, [9, 31]):
        say(f"dpd mask split {batches[:3]}")
        with Graph(0) as G:
            outs.append(run_mask_chain(G, w, masks, batches=batches)[0])
    for y in outs[1:]:
        assert np.array_equal(y.view(np.float32), outs[0].view(np.float32))


def test_fire_many_mixed_count_and_mask_instances():
    """Persistent launch and graph replay over instances of both control
    modes (B_max up to 16): equal to per-firing launches bit for bit and to
    the oracle."""
    from paper_1611_03226_amd.graph import Graph
    rng = np.random.default_rng(112)
    r, M = 192, 16
    insts = []
    for i in range(12):
        B = int(rng.integers(3, 17))
        nf = int(rng.integers(2, 7))
        mode = "mask" if i % 2 else "count"
        ctrl = _masks(rng, 2 * nf, B) if mode == "mask" else rng.integers(0, B + 1, 2 * nf).astype(np.int32)
        insts.append(dict(h=dpd_coeffs(rng, B, M), x=complex_gaussian(rng, 2 * nf * r), ctrl=ctrl, nf=nf,
                          mode=mode, hist="shared" if i % 5 == 4 else "branch"))
    res = {}
    for mode in ("per_firing", "persistent", "graph"):
        say(f"dpd mask fire_many {mode}")
        with Graph(0) as G:
            chains = []
            for d in insts:
                cap = _pow2(2 * d["nf"] * r)
                chains.append(G.dpd_chain(d["h"], r, history=d["hist"], cap_x=cap, cap_ctrl=_pow2(2 * d["nf"]),
                                          cap_y=cap, control=d["mode"]))
            for d, ch in zip(insts, chains):
                G.push(ch.x, d["x"])
                G.push(ch.ctrl, d["ctrl"])
            for _ in range(2):
                if mode == "per_firing":
                    for d, ch in zip(insts, chains):
                        for _ in range(d["nf"]):
                            G.fire(ch.actor, 1)
                else:
                    G.fire_many([c.actor for c in chains], [d["nf"] for d in insts], persistent=True,
                                graph=mode == "graph")
            ys = []
            for d, ch in zip(insts, chains):
                y = np.zeros(2 * d["nf"] * r, np.complex64)
                assert G.pop(ch.y, y) == len(y)
                ys.append(y)
            G.sync()
        res[mode] = ys
    for d, y in zip(insts, res["graph"]):
        ref = odpd.run_dpd(d["x"], d["ctrl"], d["h"], r, hist=d["hist"], control=d["mode"])
        worst, _, bad0 = rel_rms_per_firing(y, ref, r)
        assert worst <= DPD_TOL and bad0 == 0, (d["mode"], worst)
    for mode in ("persistent", "graph"):
        for a, b in zip(res["per_firing"], res[mode]):
            assert np.array_equal(a.view(np.float32), b.view(np.float32)), mode


def test_mask_validation():
    import torch
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    say("dpd mask validation")
    w = dpd_random(113, n_firings=4, r=16, n_branches_max=3, n_taps=4)
    with Graph(0) as G:
        ch = G.dpd_chain(w.h, w.r, control="mask")
        with pytest.raises(D.DFError) as e:
            G.push(ch.ctrl, np.array([8], np.int32))          # outside 0..7
        assert e.value.code == D.DF_EINVAL
        G.push(ch.ctrl, np.array([7], np.int32))               # all three branches: fine
        G.push(ch.x, w.x)
        bad = torch.tensor([9, 5, -1], dtype=torch.int32, device="cuda")
        G.push(ch.ctrl, bad)                                   # device push: checked on the device
        torch.cuda.synchronize()
        assert G.fire(ch.actor, 4) == 4
        with pytest.raises(D.DFError) as e:
            G.sync()
        assert e.value.code == D.DF_ECONTROL
        y = np.zeros(64, np.complex64)
        G.pop(ch.y, y)
    ref = odpd.run_dpd(w.x, np.array([7, 0, 5, 0]), w.h, w.r, control="mask")
    assert rel_rms_per_firing(y, ref, 16)[0] <= DPD_TOL
