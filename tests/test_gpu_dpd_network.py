"""GPU parity of the predistortion network run with materialised branch
channels (Poly -> FIR_b -> Adder, Sec. 4.2, dynamic rates of Sec. 2.2)
through the C ABI: against the FP64 oracle network per firing (relative-to-RMS
tolerance of the FP32 path), and against the fused actor body."""
import numpy as np
import pytest

from oracle import dpd as odpd
from workloads import complex_gaussian, dpd_chain, dpd_coeffs, dpd_scale

from helpers import DPD_TOL, rel_rms_per_firing, say

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _network(x, ctrl, h, r):
    import torch
    from paper_1611_03226_amd import dfhip as D
    y = torch.empty(x.shape, dtype=torch.complex64, device="cuda")
    D.df_dpd_forward_network(_t(x), _t(ctrl), _t(h), y, r)
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


@pytest.mark.parametrize("S,nf,r,B,M", [(3, 9, 64, 10, 16), (2, 17, 7, 4, 8), (1, 5, 3, 16, 4), (4, 3, 32, 1, 1)])
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
