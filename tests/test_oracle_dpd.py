"""Pins for the DPD oracle (CPU only).

The network of Sec. 4.2 (P -> FIR_b -> A, reconfigured by control tokens) is
checked against things fixed outside it: an identity configuration that must
return the read stream, library convolution / lfilter for constant control,
linearity in the coefficients, a sample-by-sample brute force on tiny graphs,
np.cumsum / np.maximum.accumulate for the rate/offset tables, and token
conservation against the control tokens.
"""
import itertools

import numpy as np
import pytest
import scipy.signal

from oracle import dpd
from workloads import dpd_chain, dpd_random


def _psi_via_abs(x, b):
    # |x|^(2b) * x through the magnitude (hypot) rather than re^2 + im^2
    return np.abs(x) ** (2 * b) * x


def test_identity_configuration_returns_read_stream_exactly():
    w = dpd_chain()
    h = np.zeros_like(w.h)
    h[0, 0] = 1.0
    y = dpd.run_dpd(w.x, w.ctrl, h, w.r, w.n_delay)
    xs = np.concatenate([np.zeros(w.n_delay), w.x.astype(np.complex128)])
    assert len(y) == w.n_firings * w.r
    assert np.array_equal(y, xs[:len(y)])        # delay tokens shift the stream by d


@pytest.mark.parametrize("B", [1, 3, 5])
def test_constant_control_equals_library_convolution(B):
    w = dpd_random(11, n_firings=12, r=32, n_branches_max=5, n_taps=7, n_delay=2,
                   ctrl=np.full(12, B))
    y = dpd.run_dpd(w.x, w.ctrl, w.h, w.r, w.n_delay)
    xs = np.concatenate([np.zeros(2), w.x.astype(np.complex128)])[:len(y)]
    want = np.zeros(len(y), np.complex128)
    for b in range(B):
        want += np.convolve(w.h[b].astype(np.complex128), _psi_via_abs(xs, b))[:len(y)]
    np.testing.assert_allclose(y, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_single_branch_equals_lfilter():
    w = dpd_random(12, n_firings=9, r=16, n_branches_max=3, n_taps=6, ctrl=np.ones(9))
    y = dpd.run_dpd(w.x, w.ctrl, w.h, w.r)
    want = scipy.signal.lfilter(w.h[0].astype(np.complex128), [1.0], w.x.astype(np.complex128))
    np.testing.assert_allclose(y, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("hist", ["branch", "shared"])
def test_linear_in_coefficients(hist):
    w = dpd_random(13, n_firings=10, r=8, n_branches_max=4, n_taps=5, ctrl_low=0)
    rng = np.random.default_rng(0)
    h2 = rng.standard_normal(w.h.shape) + 1j * rng.standard_normal(w.h.shape)
    a, b = 0.7 - 0.2j, -1.3 + 0.5j
    y1 = dpd.run_dpd(w.x, w.ctrl, w.h, w.r, hist=hist)
    y2 = dpd.run_dpd(w.x, w.ctrl, h2, w.r, hist=hist)
    y12 = dpd.run_dpd(w.x, w.ctrl, a * w.h.astype(np.complex128) + b * h2, w.r, hist=hist)
    np.testing.assert_allclose(y12, a * y1 + b * y2, rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("hist", ["branch", "shared"])
@pytest.mark.parametrize("case", [(14, 20, 8, 5, 6, 3, 0), (15, 7, 3, 4, 9, 1, 0),
                                  (16, 33, 16, 3, 4, 0, 1), (17, 5, 1, 2, 4, 2, 0)])
def test_network_equals_compacted_closed_form(hist, case):
    seed, n, r, B, M, d, lo = case
    w = dpd_random(seed, n_firings=n, r=r, n_branches_max=B, n_taps=M, n_delay=d, ctrl_low=lo)
    y = dpd.run_dpd(w.x, w.ctrl, w.h, w.r, w.n_delay, hist=hist)
    y2 = dpd.compacted_closed_form(w.x, w.ctrl, w.h, w.r, w.n_delay, hist=hist)
    scale = max(np.abs(y2).max(), 1.0)
    np.testing.assert_allclose(y, y2, rtol=0, atol=1e-12 * scale)
    xs = dpd.read_stream(w.x, w.n_delay)
    idx = np.arange(len(y))
    np.testing.assert_allclose(dpd.output_at(xs, w.ctrl, w.h, w.r, idx, hist), y,
                               rtol=0, atol=1e-12 * scale)


def _brute_force(xs, ctrl, h, r, hist):
    """Sample-at-a-time simulation: every branch keeps its own delay line of
    past basis samples, pushed one sample at a time whenever the branch is
    fed; the output sums the fed branches b < B."""
    B_max, M = h.shape
    lines = [[0j] * (M - 1) for _ in range(B_max)]
    out = []
    for j, B in enumerate(ctrl):
        for i in range(r):
            x = complex(xs[j * r + i])
            p = x.real * x.real + x.imag * x.imag
            acc = 0j
            for b in range(B_max):
                fed = hist == "shared" or b < B
                if not fed:
                    continue
                s = (p ** b) * x
                window = [s] + lines[b][::-1]          # s[t], s[t-1], ...
                u = sum(complex(h[b, m]) * window[m] for m in range(M))
                lines[b] = (lines[b] + [s])[-(M - 1):] if M > 1 else []
                if b < B:
                    acc += u
            out.append(acc)
    return np.array(out)


@pytest.mark.parametrize("hist", ["branch", "shared"])
def test_brute_force_all_short_control_sequences(hist):
    """Every control sequence of length <= 3 over B in 0..3, r in 1..3, d in 0..2."""
    rng = np.random.default_rng(5)
    h = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    for length in (1, 2, 3):
        for ctrl in itertools.product(range(4), repeat=length):
            for r in (1, 2, 3):
                for d in (0, 2):
                    x = rng.standard_normal(length * r) + 1j * rng.standard_normal(length * r)
                    y = dpd.run_dpd(x, ctrl, h, r, n_delay=d, hist=hist)
                    xs = np.concatenate([np.zeros(d), x])
                    n = min(length, len(xs) // r)
                    want = _brute_force(xs, ctrl[:n], h, r, hist)
                    np.testing.assert_allclose(y, want, rtol=1e-12, atol=1e-12)


def test_branch_and_shared_history_coincide_without_reactivation():
    w = dpd_random(18, n_firings=16, r=16, n_branches_max=5, n_taps=8,
                   ctrl=np.sort(np.random.default_rng(3).integers(0, 6, 16))[::-1])
    yb = dpd.run_dpd(w.x, w.ctrl, w.h, w.r, hist="branch")
    ys = dpd.run_dpd(w.x, w.ctrl, w.h, w.r, hist="shared")
    np.testing.assert_allclose(yb, ys, rtol=0, atol=1e-12 * np.abs(ys).max())


def test_branch_and_shared_history_differ_exactly_at_reactivations():
    ctrl = np.array([1, 3, 1, 3, 3, 1, 3])
    w = dpd_random(19, n_firings=7, r=16, n_branches_max=3, n_taps=4, ctrl=ctrl)
    yb = dpd.run_dpd(w.x, w.ctrl, w.h, w.r, hist="branch").reshape(7, 16)
    ys = dpd.run_dpd(w.x, w.ctrl, w.h, w.r, hist="shared").reshape(7, 16)
    differ = [j for j in range(7) if not np.allclose(yb[j], ys[j], rtol=0, atol=1e-12)]
    assert differ == [1, 3, 6]                    # branches 1,2 come back after a gap
    for j in differ:                               # only the first M-1 outputs change
        assert np.allclose(yb[j, 3:], ys[j, 3:], rtol=0, atol=1e-12)


@pytest.mark.parametrize("hist", ["branch", "shared"])
def test_firing_tables_and_token_conservation(hist):
    w = dpd_random(20, n_firings=40, r=8, n_branches_max=6, n_taps=3, ctrl_low=0)
    rates, offsets, prev, last = dpd.firing_tables(w.ctrl, 6, w.r, hist)
    net = dpd.DPDNetwork(w.x, w.ctrl, w.h, w.r, hist=hist)
    net.run()
    n = w.n_firings
    for b in range(6):
        fed = np.ones(n, bool) if hist == "shared" else (w.ctrl > b)
        np.testing.assert_array_equal(rates[b], np.where(w.ctrl > b, w.r, 0))
        excl = np.concatenate([[0], np.cumsum(fed)[:-1]])
        np.testing.assert_array_equal(offsets[b], w.r * excl)
        idx = np.where(fed, np.arange(n), -1)
        incl = np.maximum.accumulate(idx)
        np.testing.assert_array_equal(prev[b], np.concatenate([[-1], incl[:-1]]))
        assert last[b] == incl[-1]
        # tokens on s_b and u_b: r per feeding firing (conservation vs control)
        assert net.fs[b].n_written == w.r * fed.sum()
        assert net.fu[b].n_read == w.r * fed.sum()
    assert net.fy.n_written == n * w.r
    assert net.fx.n_read == n * w.r
    assert net.sched.blocked() == []


def test_random_schedules_identical_and_invalid_control_rejected():
    w = dpd_random(21, n_firings=12, r=8, n_branches_max=4, n_taps=5, n_delay=3, ctrl_low=0)
    ref = dpd.run_dpd(w.x, w.ctrl, w.h, w.r, w.n_delay)
    for seed in (1, 2, 3):
        y = dpd.run_dpd(w.x, w.ctrl, w.h, w.r, w.n_delay, policy="random", seed=seed)
        assert np.array_equal(y, ref)
    bad = w.ctrl.copy()
    bad[3] = 5
    with pytest.raises(ValueError):
        dpd.run_dpd(w.x, bad, w.h, w.r)
    with pytest.raises(ValueError):
        dpd.firing_tables(np.array([1, -1]), 4, 8)


def test_delay_tokens_leave_d_samples_unconsumed():
    w = dpd_chain()
    net = dpd.DPDNetwork(w.x, w.ctrl, w.h, w.r, w.n_delay)
    net.run()
    assert net.fx.count() == w.n_delay
    assert net.P.n_fired == w.n_firings


# ------------------------------------------------------------------ mask control

def test_prefix_masks_equal_branch_counts():
    w = dpd_random(41, 12, 16, 5, 4)
    masks = (1 << w.ctrl.astype(np.int64)) - 1          # B -> bits 0..B-1
    y_count = dpd.run_dpd(w.x, w.ctrl, w.h, w.r)
    y_mask = dpd.run_dpd(w.x, masks, w.h, w.r, control="mask")
    assert np.array_equal(y_count, y_mask)


def test_single_bit_masks_are_one_fir_over_its_compacted_channel():
    # only branch b ever active: the output of a firing with the bit set is
    # lfilter(h_b) of the concatenated basis samples of the active firings
    w = dpd_random(42, 10, 8, 4, 5)
    b = 2
    on = np.random.default_rng(42).random(10) < 0.6
    masks = np.where(on, 1 << b, 0)
    y = dpd.run_dpd(w.x, masks, w.h, w.r, control="mask").reshape(10, 8)
    xs = w.x.astype(np.complex128).reshape(10, 8)
    chan = np.concatenate([dpd.basis(xs[j], b) for j in range(10) if on[j]])
    u = scipy.signal.lfilter(w.h[b].astype(np.complex128), [1.0], chan).reshape(-1, 8)
    k = 0
    for j in range(10):
        if on[j]:
            assert np.allclose(y[j], u[k], rtol=0, atol=1e-12)
            k += 1
        else:
            assert not y[j].any()


def test_masks_on_disjoint_branch_sets_add():
    # branches used by m1 are never used by m2 and vice versa, so every
    # branch channel is the same in the combined network
    w = dpd_random(43, 14, 8, 6, 4)
    rng = np.random.default_rng(43)
    m1 = rng.integers(0, 64, 14) & 0b010101                  # even branches only
    m2 = rng.integers(0, 64, 14) & 0b101010                  # odd branches only
    y1 = dpd.run_dpd(w.x, m1, w.h, w.r, control="mask")
    y2 = dpd.run_dpd(w.x, m2, w.h, w.r, control="mask")
    y12 = dpd.run_dpd(w.x, m1 | m2, w.h, w.r, control="mask")
    assert np.allclose(y12, y1 + y2, rtol=0, atol=1e-12)


def test_out_of_range_mask_is_rejected():
    w = dpd_random(44, 2, 4, 3, 2)
    with pytest.raises(ValueError):
        dpd.run_dpd(w.x, np.array([1, 8]), w.h, w.r, control="mask")


@pytest.mark.parametrize("hist", ["branch", "shared"])
def test_mask_tables_against_bit_cumsums_and_network(hist):
    """Tables for mask tokens: rates = r on set bits, offsets and history
    sources = cumulative sum / maximum of the bit flags (np.cumsum,
    np.maximum.accumulate), token conservation against the mask network's
    channels, and prefix masks giving the count tables exactly."""
    rng = np.random.default_rng(45)
    w = dpd_random(45, n_firings=50, r=8, n_branches_max=6, n_taps=3)
    masks = rng.integers(0, 64, 50)
    rates, offsets, prev, last = dpd.firing_tables(masks, 6, w.r, hist, control="mask")
    net = dpd.DPDNetwork(w.x, masks, w.h, w.r, hist=hist, control="mask")
    net.run()
    n = 50
    for b in range(6):
        bit = ((masks >> b) & 1).astype(bool)
        fed = np.ones(n, bool) if hist == "shared" else bit
        np.testing.assert_array_equal(rates[b], np.where(bit, w.r, 0))
        np.testing.assert_array_equal(offsets[b], w.r * np.concatenate([[0], np.cumsum(fed)[:-1]]))
        incl = np.maximum.accumulate(np.where(fed, np.arange(n), -1))
        np.testing.assert_array_equal(prev[b], np.concatenate([[-1], incl[:-1]]))
        assert last[b] == incl[-1]
        assert net.fs[b].n_written == w.r * fed.sum()
    counts = rng.integers(0, 7, 50)
    for t_c, t_m in zip(dpd.firing_tables(counts, 6, w.r, hist),
                        dpd.firing_tables((1 << counts) - 1, 6, w.r, hist, control="mask")):
        np.testing.assert_array_equal(t_c, t_m)
