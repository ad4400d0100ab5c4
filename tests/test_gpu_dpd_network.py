"""GPU parity of the predistortion network run with materialised branch
channels (Poly -> FIR_b -> Adder, Sec. 4.2, dynamic rates of Sec. 2.2)
through the C ABI: against the FP64 oracle network per firing (relative-to-RMS
tolerance of the FP32 path), against the fused actor body, and with bit-mask
control tokens (any set of active branches)."""
import numpy as np
import pytest

from oracle import dpd as odpd
from workloads import complex_gaussian, dpd_chain, dpd_coeffs, dpd_scale

from helpers import DPD_TOL, rel_rms_per_firing, say

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _network(x, ctrl, h, r, mask=False):
    import torch
    from paper_1611_03226_amd import dfhip as D
    y = torch.empty(x.shape, dtype=torch.complex64, device="cuda")
    D.df_dpd_forward_network(_t(x), _t(ctrl), _t(h), y, r, mask=mask)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def _fused(x, ctrl, h, r):
    import torch
    from paper_1611_03226_amd import dfhip as D
    y = torch.empty(x.shape, dtype=torch.complex64, device="cuda")
    D.df_dpd_forward(_t(x), _t(ctrl), _t(h), y, r, D.DF_HIST_BRANCH)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def test_chain_workload_matches_oracle():
    say("dpd network: chain workload (64 firings of 256, B<=5, M=8)")
    w = dpd_chain()
    x = w.x[None, :]
    c = w.ctrl[None, :]
    y = _network(x, c, w.h, w.r)
    ref = odpd.run_dpd_streams(x, c, w.h, w.r, "branch")
    worst, _, bad_zero = rel_rms_per_firing(y[0], ref[0], w.r)
    print(f"worst per-firing rel error {worst:.2e}")
    assert worst <= DPD_TOL and bad_zero == 0


@pytest.mark.parametrize("S,nf,r,B,M", [(3, 9, 64, 10, 16), (2, 17, 7, 4, 8), (1, 5, 3, 16, 4), (4, 3, 32, 1, 1),
                                       (2, 4, 1500, 5, 32)])
def test_ragged_rows_match_oracle_and_fused_body(S, nf, r, B, M):
    say(f"dpd network: S={S} nf={nf} r={r} B={B} M={M}")
    rng = np.random.default_rng(S * 1000 + nf * 10 + r)
    x = complex_gaussian(rng, (S, nf * r))
    h = dpd_coeffs(rng, B, M)
    ctrl = rng.integers(0, B + 1, (S, nf)).astype(np.int32)
    ctrl[:, 0] = 0                                  # a firing with every branch at rate 0
    ctrl[0, -1] = B                                 # and one with all of them
    y = _network(x, ctrl, h, r)
    ref = odpd.run_dpd_streams(x, ctrl, h, r, "branch")
    for s in range(S):
        worst, _, bad_zero = rel_rms_per_firing(y[s], ref[s], r)
        assert worst <= DPD_TOL and bad_zero == 0, (s, worst, bad_zero)
    yf = _fused(x, ctrl, h, r)
    scale = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert np.max(np.abs(y - yf)) <= 1e-4 * scale


def test_buffers_off_16_byte_alignment():
    """Sample and output tensors starting 8 bytes past an aligned address
    (even r): the Poly and Adder passes take one sample per thread instead
    of 16-byte pairs; against the oracle and the aligned call bit for bit."""
    import torch
    from paper_1611_03226_amd import dfhip as D
    say("dpd network: buffers off 16-byte alignment")
    S, nf, r, B, M = 2, 6, 128, 7, 16
    rng = np.random.default_rng(77)
    x = complex_gaussian(rng, (S, nf * r))
    h = dpd_coeffs(rng, B, M)
    ctrl = rng.integers(0, B + 1, (S, nf)).astype(np.int32)
    xb = torch.empty(S * nf * r + 1, dtype=torch.complex64, device="cuda")
    xb[1:] = torch.from_numpy(x.reshape(-1)).cuda()
    yb = torch.empty(S * nf * r + 1, dtype=torch.complex64, device="cuda")
    xo, yo = xb[1:].view(S, nf * r), yb[1:].view(S, nf * r)
    assert xo.data_ptr() % 16 == 8 and yo.data_ptr() % 16 == 8
    D.df_dpd_forward_network(xo, _t(ctrl), _t(h), yo, r)
    torch.cuda.synchronize()
    y = yo.cpu().numpy()
    ref = odpd.run_dpd_streams(x, ctrl, h, r, "branch")
    for s in range(S):
        worst, _, bad_zero = rel_rms_per_firing(y[s], ref[s], r)
        assert worst <= DPD_TOL and bad_zero == 0
    assert np.array_equal(y.view(np.float32), _network(x, ctrl, h, r).view(np.float32))


def test_scale_workload_sampled_and_against_fused_body():
    """2^24 samples, 4096 firings of 4096, B 1..10, M 16 (the headline
    workload) through the materialised channels."""
    say("dpd network: 2^24-sample workload")
    w = dpd_scale()
    x = w.x[None, :]
    c = w.ctrl[None, :]
    y = _network(x, c, w.h, w.r)[0]
    yf = _fused(x, c, w.h, w.r)[0]
    rms = np.sqrt(np.mean(np.abs(yf.astype(np.complex128)) ** 2))
    assert np.max(np.abs(y - yf)) <= 1e-4 * rms
    idx = np.random.default_rng(3).integers(0, len(w.x), 200)
    ref = odpd.output_at(w.x, w.ctrl, w.h, w.r, idx)
    assert np.max(np.abs(y[idx] - ref)) <= DPD_TOL * rms


@pytest.mark.parametrize("S,nf,r,B,M", [(2, 21, 64, 10, 16), (3, 9, 5, 6, 6), (1, 33, 16, 16, 3)])
def test_mask_control_matches_oracle(S, nf, r, B, M):
    say(f"dpd network masks: S={S} nf={nf} r={r} B={B} M={M}")
    rng = np.random.default_rng(S * 77 + nf + B)
    x = complex_gaussian(rng, (S, nf * r))
    h = dpd_coeffs(rng, B, M)
    masks = rng.integers(0, 1 << B, (S, nf)).astype(np.int32)
    masks[:, 1] = 0
    masks[0, 2] = (1 << B) - 1
    y = _network(x, masks, h, r, mask=True)
    ref = odpd.run_dpd_streams(x, masks, h, r, "branch", control="mask")
    for s in range(S):
        worst, _, bad_zero = rel_rms_per_firing(y[s], ref[s], r)
        assert worst <= DPD_TOL and bad_zero == 0, (s, worst, bad_zero)


def test_prefix_masks_equal_counts_and_out_of_range_masks_are_zero():
    say("dpd network: prefix masks vs counts, out-of-range masks")
    rng = np.random.default_rng(78)
    S, nf, r, B, M = 2, 12, 32, 8, 8
    x = complex_gaussian(rng, (S, nf * r))
    h = dpd_coeffs(rng, B, M)
    counts = rng.integers(0, B + 1, (S, nf)).astype(np.int32)
    y_count = _network(x, counts, h, r)
    y_mask = _network(x, ((1 << counts.astype(np.int64)) - 1).astype(np.int32), h, r, mask=True)
    assert np.array_equal(y_count, y_mask)            # same channel offsets, same kernels
    bad = counts.copy()
    bad[0, 3] = 1 << B                                 # out of range: no branch active
    bad[1, 5] = -1
    y_bad = _network(x, bad, h, r, mask=True)
    fixed = bad.copy()
    fixed[0, 3] = 0
    fixed[1, 5] = 0
    assert np.array_equal(y_bad, _network(x, fixed, h, r, mask=True))
    assert not y_bad[0, 3 * r:4 * r].any()
