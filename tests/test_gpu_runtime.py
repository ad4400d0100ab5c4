"""Runtime checks on the GPU through the C ABI: the device-side ring
invariant (read <= write <= read + capacity, checked by every kernel that
advances a channel counter), the DFHIP_CHECK_INDICES debug mode, and the
binding's buffer checks against real channels."""
import numpy as np
import pytest

from helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture
def G():
    from paper_1611_03226_amd.graph import Graph
    g = Graph(0)
    yield g
    g.close()


def test_ring_invariant_violation_is_reported(G):
    """Counters driven out of range from the host: the next push's counter
    update finds write - read > capacity and df_sync reports DF_EINDEX."""
    from paper_1611_03226_amd import dfhip as D
    say("ring invariant: writer past read + capacity")
    f = D.df_fifo_create(G.g, D.DF_C64, 1, 1024)
    D.df_debug_set_counters(G.g, f, 0, 2000)
    G.push(f, np.zeros(1, np.complex64))           # host bookkeeping admits it
    with pytest.raises(D.DFError) as e:
        G.sync()
    assert e.value.code == D.DF_EINDEX


def test_ring_invariant_reader_past_writer(G):
    from paper_1611_03226_amd import dfhip as D
    say("ring invariant: reader past writer")
    f = D.df_fifo_create(G.g, D.DF_I32, 1, 64)
    G.push(f, np.arange(4, dtype=np.int32))
    D.df_debug_set_counters(G.g, f, 3, 3)          # device thinks 0 tokens are there
    out = np.zeros(4, np.int32)
    assert G.pop(f, out) == 4                       # host bookkeeping says 4
    with pytest.raises(D.DFError) as e:
        G.sync()
    assert e.value.code == D.DF_EINDEX


def test_normal_traffic_keeps_the_invariant(G):
    from paper_1611_03226_amd import dfhip as D
    say("ring invariant: wrap-around traffic")
    f = D.df_fifo_create(G.g, D.DF_I32, 1, 64)
    out = np.zeros(48, np.int32)
    for k in range(6):
        v = np.arange(48, dtype=np.int32) + 100 * k
        G.push(f, v)                                # fills the ring to 48 of 64, wraps
        assert G.pop(f, out) == 48 and np.array_equal(out, v)
    G.sync()
    assert D.df_fifo_status(G.g, f) == (288, 288, 64)


def test_check_indices_mode_reports_at_the_failing_call(monkeypatch):
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    say("DFHIP_CHECK_INDICES")
    monkeypatch.setenv("DFHIP_CHECK_INDICES", "1")
    with Graph(0) as G:
        f = D.df_fifo_create(G.g, D.DF_C64, 1, 256)
        G.push(f, np.ones(8, np.complex64))         # fine
        D.df_debug_set_counters(G.g, f, 0, 300)
        with pytest.raises(D.DFError) as e:
            G.push(f, np.ones(1, np.complex64))     # this call reports it
        assert e.value.code == D.DF_EINDEX


def test_tile_override_from_environment(monkeypatch):
    from paper_1611_03226_amd import dfhip as D
    monkeypatch.setenv("DFHIP_TILE", "bogus")
    with pytest.raises(D.DFError) as e:
        D.df_graph_create(0)
    assert e.value.code == D.DF_EINVAL
    monkeypatch.setenv("DFHIP_TILE", "512,4,2")
    g = D.df_graph_create(0)
    D.df_graph_destroy(g)


def test_binding_rejects_mismatched_buffers(G):
    import torch
    from paper_1611_03226_amd import dfhip as D
    from workloads import dpd_random
    say("binding buffer checks")
    w = dpd_random(61, n_firings=4, r=16, n_branches_max=3, n_taps=4)
    ch = G.dpd_chain(w.h, w.r)
    with pytest.raises(ValueError):
        G.push(ch.x, np.zeros(32, np.float32))                 # float pairs into a complex64 channel
    with pytest.raises(ValueError):
        G.push(ch.x, torch.zeros(32, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        G.push(ch.ctrl, np.array([1 << 33], np.int64))         # does not fit an int32 token
    G.push(ch.ctrl, np.array([1, 2, 3, 1], np.int64))          # converted, values kept
    G.push(ch.x, w.x)
    assert G.fire(ch.actor, 4) == 4
    with pytest.raises(ValueError):
        G.pop(ch.y, np.zeros(64, np.float32))
    with pytest.raises(ValueError):
        D.df_pop(G.g, ch.y, np.zeros(16, np.complex64), 64)    # no room for 64 tokens
    y = np.zeros(64, np.complex64)
    assert G.pop(ch.y, y) == 64
    assert D.df_port_rate(G.g, ch.actor, D.DF_DPD_IN) == 16
    assert D.df_port_rate(G.g, ch.actor, D.DF_DPD_CTRL) == 1
    G.sync()
    from oracle import dpd as odpd
    ref = odpd.run_dpd(w.x, np.array([1, 2, 3, 1]), w.h, w.r)
    assert np.max(np.abs(y - ref)) <= 1e-4 * np.sqrt(np.mean(np.abs(ref) ** 2))
