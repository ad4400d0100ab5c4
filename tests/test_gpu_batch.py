"""Many predistortion instances in one batch: per-actor launches, one
persistent launch, and a HIP-graph replay of the persistent chain must give
bit-identical outputs, equal to firing every instance one firing at a time,
and match the oracle."""
import numpy as np
import pytest

from oracle import dpd as odpd
from workloads import complex_gaussian, dpd_coeffs, dpd_instances

from helpers import DPD_TOL, rel_rms_per_firing, say

pytestmark = pytest.mark.gpu


def _pow2(n):
    p = 1
    while p < n:
        p <<= 1
    return p


def _instances(seed, n_inst, r, max_firings, M=16, vary_ctrl=True, B_range=(1, 10)):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_inst):
        B = int(rng.integers(B_range[0], B_range[1] + 1))
        nf = int(rng.integers(1, max_firings + 1))
        hist = "shared" if i % 5 == 4 else "branch"
        ctrl = rng.integers(0, B + 1, size=3 * nf) if vary_ctrl else np.full(3 * nf, B)
        out.append(dict(h=dpd_coeffs(rng, B, M), x=complex_gaussian(rng, 3 * nf * r),
                        ctrl=ctrl.astype(np.int32), nf=nf, hist=hist))
    return out


def _run(insts, r, mode, n_batches=3, tile=(0, 0, 0)):
    """Fire every instance nf firings per batch for n_batches batches."""
    from paper_1611_03226_amd.graph import Graph
    with Graph(0) as G:
        G.set_tile(*tile)
        chains = []
        for d in insts:
            cap = _pow2(3 * d["nf"] * r)
            ch = G.dpd_chain(d["h"], r, history=d["hist"], cap_x=cap, cap_ctrl=_pow2(3 * d["nf"]), cap_y=cap)
            chains.append(ch)
        outs = [[] for _ in insts]
        for b in range(n_batches):
            for d, ch in zip(insts, chains):
                lo, hi = b * d["nf"], (b + 1) * d["nf"]
                G.push(ch.x, d["x"][lo * r:hi * r])
                G.push(ch.ctrl, d["ctrl"][lo:hi])
            actors = [c.actor for c in chains]
            nfs = [d["nf"] for d in insts]
            if mode == "per_firing":
                for d, ch in zip(insts, chains):
                    for _ in range(d["nf"]):
                        G.fire(ch.actor, 1)
            else:
                G.fire_many(actors, nfs, persistent=mode in ("persistent", "graph"), graph=mode == "graph")
            for i, (d, ch) in enumerate(zip(insts, chains)):
                y = np.zeros(d["nf"] * r, np.complex64)
                assert G.pop(ch.y, y) == len(y)
                outs[i].append(y)
        G.sync()
    return [np.concatenate(o) for o in outs]


def test_modes_bit_identical_and_match_oracle():
    r = 256
    insts = _instances(60, 37, r, 6)
    res = {}
    for mode in ("per_firing", "many", "persistent", "graph"):
        say(f"batch mode {mode}")
        res[mode] = _run(insts, r, mode)
    for mode in ("per_firing", "graph"):
        for d, y in zip(insts, res[mode]):
            ref = odpd.run_dpd(d["x"], d["ctrl"], d["h"], r, hist=d["hist"])
            worst, _, bad0 = rel_rms_per_firing(y, ref, r)
            assert worst <= DPD_TOL and bad0 == 0, mode
    for mode in ("many", "persistent", "graph"):
        for i, (a, b) in enumerate(zip(res["per_firing"], res[mode])):
            diff = np.nonzero(a.view(np.float32) != b.view(np.float32))[0]
            assert len(diff) == 0, f"{mode} instance {i}: {len(diff)} floats differ, first at {diff[:8]} (r={r})"


@pytest.mark.parametrize("M", [16, 8, 4])
def test_wide_branch_counts_match_oracle(M):
    """Instances with n_branches_max 11..16 (the 16-branch instantiations of
    the persistent body) beside small ones, ragged r: graph replay and
    persistent launch == per-firing launches bit for bit, all against the
    oracle."""
    r = 200
    insts = _instances(63 + M, 14, r, 5, M=M, B_range=(8, 16))
    res = {}
    for mode in ("per_firing", "persistent", "graph"):
        say(f"batch B_max 11..16 M={M} {mode}")
        res[mode] = _run(insts, r, mode, 2)
    assert max(d["h"].shape[0] for d in insts) > 10
    for d, y in zip(insts, res["graph"]):
        ref = odpd.run_dpd(d["x"][:len(y)], d["ctrl"][:len(y) // r], d["h"], r, hist=d["hist"])
        worst, _, bad0 = rel_rms_per_firing(y, ref, r)
        assert worst <= DPD_TOL and bad0 == 0, (d["h"].shape, worst)
    for mode in ("persistent", "graph"):
        for a, b in zip(res["per_firing"], res[mode]):
            assert np.array_equal(a.view(np.float32), b.view(np.float32)), mode


def test_more_instances_than_a_workgroup_with_one_branch():
    """1300 single-branch instances: the persistent scan runs one wavefront
    per instance and sums more firing counts than it has threads, the order
    pass loops over the instances; graph replay == per-actor launches bit
    for bit, sampled instances against the oracle."""
    r = 64
    insts = _instances(71, 1300, r, 2, M=8, B_range=(1, 1))
    res = {}
    for mode in ("many", "graph"):
        say(f"1300 instances {mode}")
        res[mode] = _run(insts, r, mode, 2)
    for a, b in zip(res["many"], res["graph"]):
        assert np.array_equal(a.view(np.float32), b.view(np.float32))
    for d, y in list(zip(insts, res["graph"]))[::97]:
        ref = odpd.run_dpd(d["x"][:len(y)], d["ctrl"][:len(y) // r], d["h"], r, hist=d["hist"])
        worst, _, bad0 = rel_rms_per_firing(y, ref, r)
        assert worst <= DPD_TOL and bad0 == 0


@pytest.mark.parametrize("tile", [(512, 4, 2), (2048, 8, 1), (256, 4, 8), (1024, 8, 4)])
def test_tile_configurations_are_bit_identical(tile):
    r = 1024
    insts = _instances(61, 12, r, 4, vary_ctrl=True)
    say(f"batch tile {tile}")
    base = _run(insts, r, "graph", 2)
    other = _run(insts, r, "graph", 2, tile=tile)
    for a, b in zip(base, other):
        assert np.array_equal(a.view(np.float32), b.view(np.float32))


def test_lognormal_instances_full_size():
    """The 1024-instance workload (lognormal lengths 1k..256k, r = 1024):
    persistent graph replay == per-actor launches bit for bit; every
    instance against the oracle, per-firing rel-RMS."""
    from paper_1611_03226_amd.graph import Graph
    say("batch 1024 instances full size")
    w = dpd_instances()
    r = w.r
    outs = {}
    for mode in ("many", "graph"):
        with Graph(0) as G:
            chains = []
            for i in range(len(w.lengths)):
                L = int(w.lengths[i])
                ch = G.dpd_chain(w.h[i], r, cap_x=_pow2(L), cap_ctrl=_pow2(L // r), cap_y=_pow2(L))
                G.push(ch.x, w.x[i])
                G.push(ch.ctrl, w.ctrl(i))
                chains.append(ch)
            G.fire_many([c.actor for c in chains], (w.lengths // r).tolist(),
                        persistent=mode == "graph", graph=mode == "graph")
            ys = []
            for i, ch in enumerate(chains):
                y = np.zeros(int(w.lengths[i]), np.complex64)
                G.pop(ch.y, y)
                ys.append(y)
            G.sync()
        outs[mode] = ys
    for a, b in zip(outs["many"], outs["graph"]):
        assert np.array_equal(a.view(np.float32), b.view(np.float32))
    worst_all = 0.0
    for i in range(len(w.lengths)):
        ref = odpd.run_dpd(w.x[i], w.ctrl(i), w.h[i], r)
        worst, _, bad0 = rel_rms_per_firing(outs["graph"][i], ref, r)
        assert worst <= DPD_TOL and bad0 == 0, i
        worst_all = max(worst_all, worst)
    print(f"1024 instances: rel-RMS worst firing {worst_all:.3e}")


def test_fire_many_validation():
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    say("batch validation")
    rng = np.random.default_rng(1)
    with Graph(0) as G:
        a = G.dpd_chain(dpd_coeffs(rng, 3, 16), 64)
        b = G.dpd_chain(dpd_coeffs(rng, 3, 8), 64)
        with pytest.raises(D.DFError) as e:
            G.fire_many([a.actor, b.actor], [0, 0], persistent=True)     # mixed n_taps
        assert e.value.code == D.DF_EINVAL
        with pytest.raises(D.DFError) as e:
            G.fire_many([a.actor, a.actor], [0, 0])                      # duplicate
        assert e.value.code == D.DF_EINVAL
        G.push(a.x, complex_gaussian(rng, 64))
        G.push(a.ctrl, np.array([1, 2], np.int32))
        with pytest.raises(D.DFError) as e:
            G.fire_many([a.actor], [2], persistent=True)                 # 1 firing of input
        assert e.value.code == D.DF_EAGAIN
        assert G.status(a.ctrl)[:2] == (0, 2)


def test_graph_replay_with_changing_firing_counts(monkeypatch, capfd):
    """Persistent graph mode when the firing counts change between batches
    equals per-actor launches bit for bit, and the chain is captured once:
    the counts reach the replayed graph through device memory."""
    from paper_1611_03226_amd.graph import Graph
    monkeypatch.setenv("DFHIP_LOG", "1")
    r = 256
    insts = _instances(62, 10, r, 5)
    rng = np.random.default_rng(3)
    plans = [[d["nf"] for d in insts], [max(1, d["nf"] - 1) for d in insts], [d["nf"] for d in insts]]
    plans[1][0] = 0                                   # one instance idle in the second batch
    outs = {}
    capfd.readouterr()
    for mode in ("many", "graph"):
        say(f"batch changing counts {mode}")
        with Graph(0) as G:
            chains = []
            for d in insts:
                cap = _pow2(3 * d["nf"] * r)
                chains.append(G.dpd_chain(d["h"], r, history=d["hist"], cap_x=cap, cap_ctrl=_pow2(3 * d["nf"]),
                                          cap_y=cap))
            for d, ch in zip(insts, chains):
                G.push(ch.x, d["x"])
                G.push(ch.ctrl, d["ctrl"])
            ys = [[] for _ in insts]
            for nfs in plans:
                G.fire_many([c.actor for c in chains], nfs, persistent=mode == "graph", graph=mode == "graph")
                for i, (nf, ch) in enumerate(zip(nfs, chains)):
                    y = np.zeros(nf * r, np.complex64)
                    assert G.pop(ch.y, y) == len(y)
                    ys[i].append(y)
            G.sync()
        outs[mode] = [np.concatenate(v) for v in ys]
    err = capfd.readouterr().err
    assert err.count("persistent chain captured") == 1, err[-2000:]
    for a, b in zip(outs["many"], outs["graph"]):
        assert np.array_equal(a.view(np.float32), b.view(np.float32))
    for d, y in zip(insts, outs["graph"]):
        k = len(y) // r
        ref = odpd.run_dpd(d["x"][:k * r], d["ctrl"][:k], d["h"], r, hist=d["hist"])
        assert rel_rms_per_firing(y, ref, r)[0] <= DPD_TOL
