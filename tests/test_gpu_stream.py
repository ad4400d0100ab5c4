"""GPU checks of df_stream_dpd (host input copies, firings and host output
copies overlapped on three streams): bit-identical to pushing, firing and
popping each batch in turn, with rings of exactly two batches so that every
slot is reused while neighbouring batches are in flight, and with delay
tokens on the input channel."""
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


def _sequential(w, nb, n_batches, d, initial):
    from paper_1611_03226_amd.graph import Graph
    ns = nb * w.r
    with Graph(0) as G:
        ch = G.dpd_chain(w.h, w.r, d, initial, cap_x=_pow2(2 * ns + d), cap_ctrl=_pow2(2 * nb),
                         cap_y=_pow2(2 * ns))
        y = np.zeros(n_batches * ns, np.complex64)
        for k in range(n_batches):
            G.push(ch.ctrl, w.ctrl[k * nb:(k + 1) * nb])
            G.push(ch.x, w.x[k * ns:(k + 1) * ns])
            assert G.fire(ch.actor, nb) == nb
            assert G.pop(ch.y, y[k * ns:(k + 1) * ns]) == ns
        G.sync()
    return y


def _streamed(w, nb, n_batches, d, initial):
    import torch
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    ns = nb * w.r
    x = torch.from_numpy(np.ascontiguousarray(w.x[:n_batches * ns])).pin_memory().numpy()
    c = torch.from_numpy(np.ascontiguousarray(w.ctrl[:n_batches * nb])).pin_memory().numpy()
    y = torch.zeros(n_batches * ns, dtype=torch.complex64).pin_memory().numpy()
    with Graph(0) as G:
        ch = G.dpd_chain(w.h, w.r, d, initial, cap_x=_pow2(2 * ns + d), cap_ctrl=_pow2(2 * nb),
                         cap_y=_pow2(2 * ns))
        D.df_stream_dpd(G.g, ch.actor, x, c, y, n_batches, nb)
        # the channels end where the sequential form leaves them
        assert G.status(ch.y)[:2] == (n_batches * ns, n_batches * ns)
        assert G.status(ch.x)[:2] == (n_batches * ns, n_batches * ns + d)
        G.sync()
    return y


@pytest.mark.parametrize("nb,n_batches,r,B,M,d", [(8, 9, 64, 10, 16, 0), (4, 13, 32, 5, 8, 3),
                                                  (16, 5, 256, 10, 16, 0), (1, 20, 16, 4, 4, 1)])
def test_streamed_equals_sequential(nb, n_batches, r, B, M, d):
    say(f"stream_dpd nb={nb} batches={n_batches} r={r} B={B} M={M} d={d}")
    w = dpd_random(90 + nb + d, nb * n_batches, r, B, M, n_delay=d)
    initial = np.random.default_rng(5).standard_normal(d).astype(np.complex64) if d else None
    a = _sequential(w, nb, n_batches, d, initial)
    b = _streamed(w, nb, n_batches, d, initial)
    assert np.array_equal(a, b)
    # and both against the oracle network fed the same host streams
    n = nb * n_batches
    ref = odpd.run_dpd(w.x[:n * r], w.ctrl[:n], w.h, r, n_delay=d, initial=initial)
    worst, glob, bad0 = rel_rms_per_firing(b, ref, r)
    print(f"stream_dpd: rel-RMS worst firing {worst:.3e} global {glob:.3e}")
    assert worst <= DPD_TOL and bad0 == 0


def test_stream_rejects_small_channels():
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    say("stream_dpd argument checks")
    w = dpd_random(99, 8, 64, 4, 8)
    with Graph(0) as G:
        ch = G.dpd_chain(w.h, w.r, cap_x=512, cap_ctrl=64, cap_y=512)   # one batch of 8 x 64 only
        y = np.zeros(8 * 64, np.complex64)
        with pytest.raises(D.DFError) as e:
            D.df_stream_dpd(G.g, ch.actor, np.ascontiguousarray(w.x), np.ascontiguousarray(w.ctrl), y, 1, 8)
        assert e.value.code == D.DF_EINVAL
