"""The matrix-core form of the 16-tap predistortion body (DFHIP_BODY=mx):
per block of 16 samples and chunk of four branches one v_mfma_f32_16x16x4_f32
gives the tap polynomials (Sec. 4.2 Poly feeding the FIR filters, as the
power-basis sum), the VALU takes the complex products and the diagonal sum.
It rounds differently from the VALU form, so it is checked against the
oracle (per-firing rel-RMS), and its paths (single actor, persistent batch,
stateless rows) against each other bit for bit."""
import numpy as np
import pytest

from oracle import dpd as odpd
from workloads import complex_gaussian, dpd_coeffs, dpd_random, dpd_scale

from helpers import DPD_TOL, rel_rms_per_firing, run_dpd_chain, say

pytestmark = pytest.mark.gpu


@pytest.fixture
def mx(monkeypatch):
    monkeypatch.setenv("DFHIP_BODY", "mx")


def _pow2(n):
    p = 1
    while p < n:
        p <<= 1
    return p


CASES = [
    # seed, n, r, B_max, M, d, ctrl_low, hist, batches, cap_x
    (301, 24, 64, 5, 16, 3, 0, "branch", [5, 1, 9, 9], 1024),   # ring wrap, zero control, tile of 64
    (302, 30, 100, 6, 16, 1, 0, "branch", [7, 7, 16], 4096),     # r not a multiple of 16
    (303, 12, 2000, 10, 16, 2, 1, "shared", [12], 0),            # several tiles per firing, ragged last
    (304, 20, 300, 13, 16, 0, 0, "branch", [20], 0),             # four branch chunks
    (305, 16, 257, 16, 16, 4, 0, "branch", [3, 13], 8192),       # B_max 16, delay tokens
]


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}" for c in CASES])
def test_mx_random_cases_match_oracle(mx, case):
    from paper_1611_03226_amd.graph import Graph
    seed, n, r, B, M, d, lo, hist, batches, cap = case
    say(f"mx body case {case}")
    w = dpd_random(seed, n_firings=n, r=r, n_branches_max=B, n_taps=M, n_delay=d, ctrl_low=lo)
    with Graph(0) as G:
        y, _ = run_dpd_chain(G, w, hist=hist, batches=batches, cap_x=cap)
    ref = odpd.run_dpd(w.x, w.ctrl, w.h, w.r, w.n_delay, hist=hist)
    worst, glob, bad0 = rel_rms_per_firing(y, ref, r)
    print(f"mx case {seed}: worst {worst:.3e} global {glob:.3e}")
    assert worst <= DPD_TOL and bad0 == 0


def test_mx_masks_and_identity(mx):
    """Bit-mask control tokens (non-prefix branch sets) and the identity
    configuration (bit-exact: one unit coefficient)."""
    from paper_1611_03226_amd.graph import Graph
    say("mx body masks")
    rng = np.random.default_rng(310)
    n, r, B = 40, 96, 12
    w = dpd_random(310, n_firings=n, r=r, n_branches_max=B, n_taps=16)
    masks = rng.integers(0, 1 << B, n).astype(np.int32)
    with Graph(0) as G:
        ch = G.dpd_chain(w.h, r, cap_x=_pow2(n * r), cap_ctrl=64, cap_y=_pow2(n * r), control="mask")
        G.push(ch.x, w.x)
        G.push(ch.ctrl, masks)
        assert G.fire(ch.actor, n) == n
        y = np.zeros(n * r, np.complex64)
        G.pop(ch.y, y)
    ref = odpd.run_dpd(w.x, masks, w.h, r, control="mask")
    assert rel_rms_per_firing(y, ref, r)[0] <= DPD_TOL
    w2 = dpd_random(311, n_firings=8, r=64, n_branches_max=3, n_taps=16, ctrl_low=1)
    w2.h[:] = 0
    w2.h[0, 0] = 1
    with Graph(0) as G:
        y2, _ = run_dpd_chain(G, w2)
    assert np.array_equal(y2.view(np.float32), w2.x.view(np.float32))


def test_mx_persistent_and_per_actor_bit_identical(mx):
    """Uneven instances through df_fire_many (persistent graph) and one
    df_fire per actor: the same matrix-core tiles, bit-identical outputs."""
    from paper_1611_03226_amd.graph import Graph
    say("mx body persistent vs per actor")
    rng = np.random.default_rng(320)
    r = 512
    insts = []
    for i in range(12):
        B = int(rng.integers(1, 11))
        nf = int(rng.integers(1, 7))
        insts.append(dict(h=dpd_coeffs(rng, B, 16), x=complex_gaussian(rng, nf * r),
                          ctrl=rng.integers(0, B + 1, nf).astype(np.int32), nf=nf))
    outs = {}
    for mode in ("actor", "graph"):
        with Graph(0) as G:
            chains = []
            for d in insts:
                ch = G.dpd_chain(d["h"], r, cap_x=_pow2(d["nf"] * r), cap_ctrl=8, cap_y=_pow2(d["nf"] * r))
                G.push(ch.x, d["x"])
                G.push(ch.ctrl, d["ctrl"])
                chains.append(ch)
            if mode == "actor":
                for d, ch in zip(insts, chains):
                    G.fire(ch.actor, d["nf"])
            else:
                G.fire_many([c.actor for c in chains], [d["nf"] for d in insts], persistent=True, graph=True)
            ys = []
            for d, ch in zip(insts, chains):
                y = np.zeros(d["nf"] * r, np.complex64)
                G.pop(ch.y, y)
                ys.append(y)
        outs[mode] = ys
    for d, a, b in zip(insts, outs["actor"], outs["graph"]):
        assert np.array_equal(a.view(np.float32), b.view(np.float32))
        ref = odpd.run_dpd(d["x"], d["ctrl"], d["h"], r)
        assert rel_rms_per_firing(a, ref, r)[0] <= DPD_TOL


def test_mx_stateless_rows_match_oracle(mx):
    import torch
    from paper_1611_03226_amd import dfhip as D
    say("mx body stateless rows")
    rng = np.random.default_rng(330)
    S, L, r, B = 6, 4096, 256, 10
    x = complex_gaussian(rng, S * L).reshape(S, L)
    ctrl = rng.integers(0, B + 1, (S, L // r)).astype(np.int32)
    h = dpd_coeffs(rng, B, 16)
    y = torch.empty((S, L), dtype=torch.complex64, device="cuda")
    D.df_dpd_forward(torch.from_numpy(x).cuda(), torch.from_numpy(ctrl).cuda(), torch.from_numpy(h).cuda(), y, r,
                     D.DF_HIST_BRANCH)
    torch.cuda.synchronize()
    ref = odpd.run_dpd_streams(x, ctrl, h, r, "branch")
    for s in range(S):
        worst, _, bad0 = rel_rms_per_firing(y[s].cpu().numpy(), ref[s], r)
        assert worst <= DPD_TOL and bad0 == 0


def test_mx_scale_workload_reduced_length(mx):
    from paper_1611_03226_amd.graph import Graph
    say("mx body scale 2^20")
    w = dpd_scale(n_samples=1 << 20)
    with Graph(0) as G:
        y, _ = run_dpd_chain(G, w)
    ref = odpd.run_dpd(w.x, w.ctrl, w.h, w.r)
    worst, glob, bad0 = rel_rms_per_firing(y, ref, w.r)
    print(f"mx scale 2^20: worst {worst:.3e} global {glob:.3e}")
    assert worst <= DPD_TOL and bad0 == 0
