"""The scan of the next batch run ahead (Sec. 2.2: a firing's rates depend
only on its control token, so the control intake of batch k+1 can run
while batch k computes).  Batches fired with their control tokens already
in the channel must match the oracle and be bit-identical to the same
batches with run-ahead switched off (DFHIP_SCAN_AHEAD=0); a scan that
assumed the wrong batch is discarded; a bad token in a batch scanned ahead
is reported with that batch, not before it."""
import re

import numpy as np
import pytest

from oracle import dpd as odpd
from workloads import dpd_random

from helpers import DPD_TOL, rel_rms_per_firing, say

pytestmark = pytest.mark.gpu


def _pow2(n):
    p = 1
    while p < n:
        p <<= 1
    return p


def _ahead(log, what):
    """Lines of the library's log (DFHIP_LOG=2) about scans run ahead."""
    return len(re.findall(rf"\[dfhip\] scan run ahead for \d+ firings at \d+ {what}", log))


def _masks(rng, n, B):
    m = rng.integers(1, 1 << B, n)
    m[rng.random(n) < 0.1] = 0
    return m.astype(np.int32)


def run_ahead_chain(w, ctrl, batches, hist="branch", control="count", lead=None, cap_ctrl=0, ahead=True,
                    monkeypatch=None):
    """All samples pushed first; control tokens pushed `lead` batches ahead of
    the firing (all at once when None); the batches fired one by one."""
    from paper_1611_03226_amd.graph import Graph
    monkeypatch.setenv("DFHIP_SCAN_AHEAD", "1" if ahead else "0")
    n = sum(batches)
    bounds = np.cumsum([0] + list(batches))
    with Graph(0) as G:
        ch = G.dpd_chain(w.h, w.r, w.n_delay, history=hist, cap_x=_pow2(n * w.r + w.n_delay),
                         cap_ctrl=cap_ctrl or _pow2(n), cap_y=_pow2(max(batches) * w.r), control=control)
        G.push(ch.x, w.x)
        pushed = 0
        out = []
        for i, k in enumerate(batches):
            upto = n if lead is None else bounds[min(i + 1 + lead, len(batches))]
            if upto > pushed:
                G.push(ch.ctrl, np.ascontiguousarray(ctrl[pushed:upto]))
                pushed = upto
            assert G.fire(ch.actor, k) == k
            buf = np.zeros(k * w.r, np.complex64)
            assert G.pop(ch.y, buf) == k * w.r
            out.append(buf)
        G.sync()
    return np.concatenate(out)


CASES = [
    # seed, batches, B_max, M, hist, control
    (201, [300] * 4, 10, 16, "branch", "count"),
    (202, [300, 300, 200, 200, 300, 65, 65], 10, 16, "shared", "count"),   # sizes change: scans discarded
    (203, [257] * 3, 13, 8, "branch", "mask"),
    (204, [100, 100, 100], 16, 4, "branch", "mask"),
    (205, [4096, 4096], 10, 16, "branch", "count"),
]


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}" for c in CASES])
def test_run_ahead_matches_oracle_and_serial_scan(case, monkeypatch, capfd):
    seed, batches, B, M, hist, control = case
    say(f"scan ahead {case[:2]}")
    rng = np.random.default_rng(seed)
    n = sum(batches)
    r = 64 if n < 5000 else 16
    w = dpd_random(seed, n_firings=n, r=r, n_branches_max=B, n_taps=M, n_delay=2, ctrl_low=0)
    ctrl = _masks(rng, n, B) if control == "mask" else w.ctrl
    monkeypatch.setenv("DFHIP_LOG", "2")
    y = run_ahead_chain(w, ctrl, batches, hist, control, monkeypatch=monkeypatch)
    log = capfd.readouterr().err
    y0 = run_ahead_chain(w, ctrl, batches, hist, control, ahead=False, monkeypatch=monkeypatch)
    ref = odpd.run_dpd(w.x, ctrl, w.h, w.r, w.n_delay, hist=hist, control=control)
    worst, glob, bad0 = rel_rms_per_firing(y, ref, w.r)
    print(f"scan ahead {seed}: worst {worst:.3e} global {glob:.3e}")
    assert worst <= DPD_TOL and bad0 == 0
    assert np.array_equal(y.view(np.float32), y0.view(np.float32))
    # after batch i (over 64 firings), a scan of the next batch of its size
    # runs ahead when that many tokens remain; the next batch uses it if it
    # has that size, else discards it
    used = discarded = 0
    left = n
    for a, b in zip(batches, batches[1:]):
        left -= a
        if a > 64 and left >= a:
            used += a == b
            discarded += a != b
    assert _ahead(log, "used") == used
    assert _ahead(log, "discarded") == discarded


@pytest.mark.parametrize("lead", [1, 2])
def test_run_ahead_with_control_ring_wrap(lead, monkeypatch):
    """Control tokens pushed one or two batches ahead into a ring of
    (lead + 1) batches: the scan run ahead reads across the wrap."""
    say(f"scan ahead wrap lead={lead}")
    batches = [96] * 7
    n = sum(batches)
    w = dpd_random(210 + lead, n_firings=n, r=32, n_branches_max=10, n_taps=16, ctrl_low=0)
    cap = _pow2((lead + 1) * 96)
    y = run_ahead_chain(w, w.ctrl, batches, lead=lead, cap_ctrl=cap, monkeypatch=monkeypatch)
    y0 = run_ahead_chain(w, w.ctrl, batches, lead=lead, cap_ctrl=cap, ahead=False, monkeypatch=monkeypatch)
    ref = odpd.run_dpd(w.x, w.ctrl, w.h, w.r)
    assert rel_rms_per_firing(y, ref, w.r)[0] <= DPD_TOL
    assert np.array_equal(y.view(np.float32), y0.view(np.float32))


def test_tables_of_a_batch_scanned_ahead(monkeypatch):
    """Rates, offsets and history sources of the last batch (scanned ahead)
    are bit-exact against the oracle's tables of that batch."""
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    say("scan ahead tables")
    monkeypatch.setenv("DFHIP_SCAN_AHEAD", "1")
    k, nb = 200, 3
    w = dpd_random(220, n_firings=k * nb, r=16, n_branches_max=7, n_taps=8, ctrl_low=0)
    with Graph(0) as G:
        ch = G.dpd_chain(w.h, w.r, cap_x=_pow2(k * nb * w.r), cap_ctrl=1024, cap_y=_pow2(k * w.r))
        G.push(ch.x, w.x)
        G.push(ch.ctrl, w.ctrl)
        buf = np.zeros(k * w.r, np.complex64)
        for _ in range(nb):
            assert G.fire(ch.actor, k) == k
            G.pop(ch.y, buf)
        rates, offs, prev = D.df_debug_last_batch(G.g, ch.actor, 7, k)
    r_ref, o_ref, p_ref, _ = odpd.firing_tables(w.ctrl[-k:], 7, w.r, "branch")
    assert np.array_equal(rates, r_ref)
    assert np.array_equal(offs, o_ref)
    assert np.array_equal(prev, p_ref)


@pytest.mark.parametrize("second", [100, 60])
def test_bad_token_reported_with_its_batch(second, monkeypatch):
    """A device-pushed out-of-range token in the second batch: the first
    batch's sync reports nothing (the scan run ahead keeps its error apart),
    the second batch's sync reports DF_ECONTROL, whether the second batch
    uses the scan run ahead (same size) or discards it (60 firings)."""
    import torch
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    say(f"scan ahead bad token second={second}")
    monkeypatch.setenv("DFHIP_SCAN_AHEAD", "1")
    w = dpd_random(230, n_firings=200, r=16, n_branches_max=5, n_taps=16, ctrl_low=0)
    ctrl = w.ctrl.copy()
    ctrl[100 + 17] = 9                                   # outside 0..5
    with Graph(0) as G:
        ch = G.dpd_chain(w.h, w.r, cap_x=4096, cap_ctrl=256, cap_y=2048)
        G.push(ch.x, w.x)
        G.push(ch.ctrl, torch.from_numpy(ctrl).cuda())  # validated on the device only
        torch.cuda.synchronize()
        buf = np.zeros(100 * w.r, np.complex64)
        assert G.fire(ch.actor, 100) == 100
        G.sync()                                         # batch 1 is clean
        G.pop(ch.y, buf)
        ref = odpd.run_dpd(w.x[:1600], w.ctrl[:100], w.h, w.r)
        assert rel_rms_per_firing(buf, ref, w.r)[0] <= DPD_TOL
        assert G.fire(ch.actor, second) == second
        with pytest.raises(D.DFError) as e:
            G.sync()
        assert e.value.code == D.DF_ECONTROL


def test_scan_ahead_discarded_after_other_firing_paths(monkeypatch, capfd):
    """df_fire leaves a scan of the next 200 firings behind.  df_fire_many
    per actor fires through the same path and uses it; the persistent batch
    consumes the tokens its own way, so the next df_fire starts elsewhere
    and must discard the stale scan.  Outputs against the oracle over the
    whole sequence."""
    from paper_1611_03226_amd.graph import Graph
    say("scan ahead discarded after fire_many")
    monkeypatch.setenv("DFHIP_SCAN_AHEAD", "1")
    monkeypatch.setenv("DFHIP_LOG", "2")
    batches = [("fire", 200), ("many", 200), ("fire", 200), ("pers", 200), ("fire", 200), ("fire", 200)]
    n = sum(k for _, k in batches)
    w = dpd_random(240, n_firings=n, r=32, n_branches_max=10, n_taps=16, ctrl_low=0)
    out = []
    with Graph(0) as G:
        ch = G.dpd_chain(w.h, w.r, cap_x=_pow2(n * w.r), cap_ctrl=_pow2(n), cap_y=_pow2(200 * w.r))
        G.push(ch.x, w.x)
        G.push(ch.ctrl, w.ctrl)
        for mode, k in batches:
            if mode == "fire":
                assert G.fire(ch.actor, k) == k
            else:
                G.fire_many([ch.actor], [k], persistent=mode == "pers")
            buf = np.zeros(k * w.r, np.complex64)
            assert G.pop(ch.y, buf) == k * w.r
            out.append(buf)
        G.sync()
    log = capfd.readouterr().err
    y = np.concatenate(out)
    ref = odpd.run_dpd(w.x, w.ctrl, w.h, w.r)
    assert rel_rms_per_firing(y, ref, w.r)[0] <= DPD_TOL
    # scans run ahead after the first, third and fifth batch (df_fire only):
    # the per-actor df_fire_many uses the first, the persistent batch skips
    # the second (discarded by the fifth batch), the sixth uses the third
    assert _ahead(log, "discarded") == 1
    assert _ahead(log, "used") == 2
