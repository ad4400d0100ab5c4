"""GPU parity of the predistortion actor through the C ABI against the FP64
oracle network: rate/offset tables and channel indices bit-exact, outputs
within 1e-4 relative-to-RMS per firing, identity configuration bit-exact,
batching and batch splits bit-identical."""
import itertools

import numpy as np
import pytest

from oracle import dpd as odpd
from workloads import dpd_chain, dpd_random, dpd_scale

from helpers import DPD_TOL, rel_rms_per_firing, run_dpd_chain, say

pytestmark = pytest.mark.gpu


@pytest.fixture
def G():
    from paper_1611_03226_amd.graph import Graph
    g = Graph(0)
    yield g
    g.close()


def test_chain_workload_matches_oracle(G):
    say("dpd chain 64x256 B5 M8 d4")
    w = dpd_chain()
    y, ch = run_dpd_chain(G, w)
    ref = odpd.run_dpd(w.x, w.ctrl, w.h, w.r, w.n_delay)
    worst, glob, bad0 = rel_rms_per_firing(y, ref, w.r)
    print(f"dpd chain rel-RMS worst firing {worst:.3e} global {glob:.3e}")
    assert worst <= DPD_TOL and bad0 == 0
    # indices: 64 firings consumed 64 control tokens and 16384 of the 16388
    # read-stream tokens; 4 input tokens are left (the 4 delay tokens' shift)
    assert G.status(ch.ctrl)[:2] == (64, 64)
    assert G.status(ch.x)[:2] == (16384, 16388)
    assert G.status(ch.y)[:2] == (16384, 16384)
    G.sync()


def test_identity_configuration_is_bit_exact(G):
    say("dpd identity")
    w = dpd_chain()
    w.h[:] = 0
    w.h[0, 0] = 1
    y, _ = run_dpd_chain(G, w)
    xs = np.concatenate([np.zeros(w.n_delay, np.complex64), w.x])[:len(y)]
    assert np.array_equal(y.view(np.float32), xs.view(np.float32))


@pytest.mark.parametrize("hist", ["branch", "shared"])
def test_rate_offset_tables_bit_exact(G, hist):
    say(f"dpd tables {hist}")
    from paper_1611_03226_amd import dfhip as D
    w = dpd_random(40, n_firings=300, r=16, n_branches_max=7, n_taps=8, ctrl_low=0)
    y, ch = run_dpd_chain(G, w, hist=hist)
    rates, offs, prev = D.df_debug_last_batch(G.g, ch.actor, 7, 300)
    r_ref, o_ref, p_ref, _ = odpd.firing_tables(w.ctrl, 7, w.r, hist)
    assert np.array_equal(rates, r_ref)
    assert np.array_equal(offs, o_ref)
    assert np.array_equal(prev, p_ref)
    ref = odpd.run_dpd(w.x, w.ctrl, w.h, w.r, hist=hist)
    assert rel_rms_per_firing(y, ref, w.r)[0] <= DPD_TOL


CASES = [
    # seed, n, r, B_max, M, d, ctrl_low, hist, batches, cap_x
    (41, 24, 64, 5, 8, 3, 0, "branch", [5, 1, 9, 9], 1024),  # ring wrap, zero control
    (42, 30, 100, 6, 16, 1, 0, "branch", [7, 7, 16], 2048),  # r not a tile multiple, wrap
    (43, 16, 1030, 10, 16, 0, 1, "shared", [3, 13], 0),      # ragged tail tile
    (44, 20, 9, 4, 5, 2, 0, "branch", [20], 256),            # generic kernel (M=5)
    (45, 12, 40, 3, 4, 0, 0, "shared", [1] * 12, 64),        # M=4 tiled, per-firing
    (46, 40, 31, 16, 32, 0, 0, "branch", [11, 29], 0),       # B_max 16, M 32 (generic)
    (47, 33, 2048, 10, 16, 4, 0, "branch", [33], 0),         # tiles of 1024 in a firing
    (48, 9, 15, 2, 16, 0, 0, "branch", [4, 5], 128),         # r = M - 1 exactly, wrap
    # n_branches_max 11..16: the tiled kernels' 16-branch instantiations
    (70, 24, 300, 11, 16, 2, 0, "branch", [6, 6, 6, 6], 2048),  # B_max 11, M 16, ragged tile, wrap
    (71, 20, 1100, 13, 16, 0, 1, "shared", [20], 0),         # B_max 13, M 16, ragged tail tile
    (72, 32, 257, 16, 16, 3, 0, "branch", [5, 27], 8192),    # B_max 16, M 16, delay, wrap
    (73, 28, 96, 16, 8, 1, 0, "branch", [10, 9, 9], 1024),   # B_max 16, M 8, wrap
    (74, 36, 70, 13, 8, 0, 0, "shared", [9, 9, 18], 0),      # B_max 13, M 8
    (75, 40, 50, 16, 4, 2, 0, "branch", [13, 14, 13], 1024), # B_max 16, M 4, wrap
    (76, 30, 33, 11, 4, 0, 1, "branch", [1] * 30, 64),       # B_max 11, M 4, per-firing
]


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}" for c in CASES])
def test_random_cases_match_oracle(G, case):
    seed, n, r, B, M, d, lo, hist, batches, cap = case
    say(f"dpd case {case}")
    w = dpd_random(seed, n_firings=n, r=r, n_branches_max=B, n_taps=M, n_delay=d, ctrl_low=lo)
    y, _ = run_dpd_chain(G, w, hist=hist, batches=batches, cap_x=cap)
    ref = odpd.run_dpd(w.x, w.ctrl, w.h, w.r, w.n_delay, hist=hist)
    worst, glob, bad0 = rel_rms_per_firing(y, ref, r)
    print(f"case {seed}: worst {worst:.3e} global {glob:.3e}")
    assert worst <= DPD_TOL and bad0 == 0


@pytest.mark.parametrize("hist", ["branch", "shared"])
def test_batched_equals_per_firing_and_splits(hist):
    """1 x 64 == 64 x 1 == 8 x 8 (bit-identical), on fresh graphs."""
    from paper_1611_03226_amd.graph import Graph
    w = dpd_random(50, n_firings=64, r=128, n_branches_max=6, n_taps=8, n_delay=2, ctrl_low=0)
    outs = []
    for batches in ([64], [1] * 64, [8] * 8, [3, 29, 1, 31]):
        say(f"dpd split {hist} {batches[:3]}")
        with Graph(0) as G:
            y, _ = run_dpd_chain(G, w, hist=hist, batches=batches)
        outs.append(y)
    for y in outs[1:]:
        assert np.array_equal(y.view(np.float32), outs[0].view(np.float32))


def test_run_twice_is_deterministic(G):
    from paper_1611_03226_amd.graph import Graph
    w = dpd_random(51, n_firings=40, r=512, n_branches_max=10, n_taps=16, ctrl_low=1)
    say("dpd determinism")
    y1, _ = run_dpd_chain(G, w)
    with Graph(0) as G2:
        y2, _ = run_dpd_chain(G2, w)
    assert np.array_equal(y1.view(np.float32), y2.view(np.float32))


@pytest.mark.parametrize("hist", ["branch", "shared"])
def test_brute_force_short_control_sequences(hist):
    """Every control sequence of length <= 3 over B in 0..3, r in {1, 3, 7},
    d in {0, 2}; each sequence on its own actor (zero initial state)."""
    from paper_1611_03226_amd.graph import Graph
    rng = np.random.default_rng(7)
    h = (rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))).astype(np.complex64)
    seqs = [s for L in (1, 2, 3) for s in itertools.product(range(4), repeat=L)]
    for r in (2, 3, 7):
        for d in (0, 2):
            say(f"dpd brute force {hist} r={r} d={d}")
            with Graph(0) as G:
                chains = []
                for s in seqs:
                    x = (rng.standard_normal(len(s) * r) + 1j * rng.standard_normal(len(s) * r)).astype(np.complex64)
                    ch = G.dpd_chain(h, r, d, history=hist, cap_x=64, cap_ctrl=64, cap_y=64)
                    G.push(ch.x, x)
                    G.push(ch.ctrl, np.array(s, np.int32))
                    chains.append((s, x, ch))
                for s, x, ch in chains:
                    n = min(len(s), (len(x) + d) // r)
                    assert G.fire(ch.actor, n) == n
                for s, x, ch in chains:
                    n = min(len(s), (len(x) + d) // r)
                    y = np.zeros(n * r, np.complex64)
                    assert G.pop(ch.y, y) == n * r
                    ref = odpd.run_dpd(x, s, h, r, n_delay=d, hist=hist)
                    np.testing.assert_allclose(y, ref, rtol=1e-5, atol=1e-5 * max(1, np.abs(ref).max()))


def test_admission_is_all_or_nothing(G):
    from paper_1611_03226_amd import dfhip as D
    say("dpd admission")
    w = dpd_random(52, n_firings=8, r=32, n_branches_max=3, n_taps=4)
    ch = G.dpd_chain(w.h, w.r, cap_x=256, cap_ctrl=16, cap_y=128)
    G.push(ch.x, w.x[:5 * 32])
    G.push(ch.ctrl, w.ctrl[:8])
    with pytest.raises(D.DFError) as e:
        G.fire(ch.actor, 6)                    # only 5 firings of input
    assert e.value.code == D.DF_EAGAIN
    assert G.status(ch.ctrl)[:2] == (0, 8)     # nothing consumed
    assert G.fire(ch.actor, 6, partial=True) == 4   # output space: 128 / 32
    with pytest.raises(D.DFError) as e:
        G.push(ch.ctrl, np.array([4], np.int32))   # outside 0..3
    assert e.value.code == D.DF_EINVAL
    with pytest.raises(D.DFError) as e:
        G.push(ch.y, np.zeros(4, np.complex64))    # an actor writes y
    assert e.value.code == D.DF_ESTATE
    G.sync()


def test_device_control_out_of_range_is_sticky(G):
    import torch
    from paper_1611_03226_amd import dfhip as D
    say("dpd device control error")
    w = dpd_random(53, n_firings=4, r=16, n_branches_max=3, n_taps=4)
    ch = G.dpd_chain(w.h, w.r)
    G.push(ch.x, w.x)
    bad = torch.tensor([1, 9, 2, 3], dtype=torch.int32, device="cuda")
    G.push(ch.ctrl, bad)                       # device push: validated on the device
    torch.cuda.synchronize()
    assert G.fire(ch.actor, 4) == 4
    with pytest.raises(D.DFError) as e:
        G.sync()
    assert e.value.code == D.DF_ECONTROL
    y = np.zeros(64, np.complex64)
    G.pop(ch.y, y)
    ctrl = np.array([1, 0, 2, 3])              # the bad token acts as 0
    ref = odpd.run_dpd(w.x, ctrl, w.h, w.r)
    assert rel_rms_per_firing(y, ref, 16)[0] <= DPD_TOL


def test_scale_workload_reduced_length(G):
    say("dpd scale 2^18")
    w = dpd_scale(n_samples=1 << 18)
    y, _ = run_dpd_chain(G, w)
    ref = odpd.run_dpd(w.x, w.ctrl, w.h, w.r)
    worst, glob, _ = rel_rms_per_firing(y, ref, w.r)
    print(f"dpd scale 2^18: worst {worst:.3e} global {glob:.3e}")
    assert worst <= DPD_TOL


def test_scale_workload_full_size(G):
    """2^24 samples in one 4096-firing batch, in the launch configuration the
    benchmark times; every firing against the FP64 oracle network."""
    say("dpd scale 2^24 full")
    w = dpd_scale()
    y, ch = run_dpd_chain(G, w, cap_x=1 << 24, cap_ctrl=4096, cap_y=1 << 24)
    ref = odpd.run_dpd(w.x, w.ctrl, w.h, w.r)
    worst, glob, bad0 = rel_rms_per_firing(y, ref, w.r)
    print(f"dpd scale 2^24: rel-RMS worst firing {worst:.3e} global {glob:.3e}")
    assert worst <= DPD_TOL and bad0 == 0


@pytest.mark.parametrize("hist", ["branch", "shared"])
def test_tables_and_outputs_many_firings(G, hist):
    """A batch of 9000 firings: the scan takes three passes of 4096 firings
    with carries, the grouped order is rebuilt from memory; tables bit-exact,
    outputs within tolerance."""
    from paper_1611_03226_amd import dfhip as D
    say(f"dpd 9000 firings {hist}")
    n = 9000
    w = dpd_random(55, n_firings=n, r=16, n_branches_max=7, n_taps=8, ctrl_low=0)
    y, ch = run_dpd_chain(G, w, hist=hist)
    rates, offs, prev = D.df_debug_last_batch(G.g, ch.actor, 7, n)
    r_ref, o_ref, p_ref, _ = odpd.firing_tables(w.ctrl, 7, w.r, hist)
    assert np.array_equal(rates, r_ref)
    assert np.array_equal(offs, o_ref)
    assert np.array_equal(prev, p_ref)
    ref = odpd.run_dpd(w.x, w.ctrl, w.h, w.r, hist=hist)
    worst, _, bad0 = rel_rms_per_firing(y, ref, w.r)
    assert worst <= DPD_TOL and bad0 == 0
