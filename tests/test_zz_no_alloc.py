"""The allocation-free forward entry point (df_dpd_forward_noalloc) against
df_dpd_forward through the C ABI: identical outputs on two calls in a row
(the second smaller, so stale scratch from the first would show), with and
without control tokens, and the size limit."""
import numpy as np
import pytest

from workloads import complex_gaussian, dpd_coeffs

from helpers import say

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("with_ctrl,hist", [(True, 0), (True, 1), (False, 0)])
def test_noalloc_forward_equals_forward_twice(with_ctrl, hist):
    import torch
    from paper_1611_03226_amd import dfhip as D
    rng = np.random.default_rng(300 + hist + 2 * with_ctrl)
    for S, nf, r, B, M in ((4, 96, 512, 10, 16), (2, 13, 100, 7, 8)):
        say(f"no-alloc forward ctrl={with_ctrl} hist={hist} S={S} nf={nf} r={r} B={B} M={M}")
        L = nf * r
        x = _t(complex_gaussian(rng, (S, L)))
        h = _t(dpd_coeffs(rng, B, M))
        ctrl = _t(rng.integers(0, B + 1, (S, nf)).astype(np.int32)) if with_ctrl else None
        y0 = torch.zeros((S, L), dtype=torch.complex64, device="cuda")
        y1 = torch.full((S, L), float("nan"), dtype=torch.complex64, device="cuda")
        D.df_dpd_forward(x, ctrl, h, y0, r, hist)
        D.df_dpd_forward_noalloc(x, ctrl, h, y1, r, hist)
        torch.cuda.synchronize()
        a = torch.view_as_real(y0).cpu().numpy()
        b = torch.view_as_real(y1).cpu().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_noalloc_rejects_calls_beyond_its_scratch():
    import torch
    from paper_1611_03226_amd import dfhip as D
    say("no-alloc size limit")
    assert D.df_dpd_forward_noalloc_max_bytes() == 12 << 20
    S, nf, r, B, M = 1, 40000, 32, 16, 32                      # 40000 firings: beyond the array
    x = torch.zeros((S, nf * r), dtype=torch.complex64, device="cuda")
    y = torch.zeros_like(x)
    h = torch.zeros((B, M), dtype=torch.complex64, device="cuda")
    c = torch.ones((S, nf), dtype=torch.int32, device="cuda")
    with pytest.raises(D.DFError) as e:
        D.df_dpd_forward_noalloc(x, c, h, y, r)
    assert e.value.code == D.DF_EINVAL
