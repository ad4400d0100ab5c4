"""GPU parity of the stateless predistortion forward, the memory-polynomial
input adjoint, the coefficient adjoint and the autograd functions, against
the FP64 oracle (and finite differences of the GPU forward)."""
import numpy as np
import pytest

from oracle import dpd as odpd
from oracle import pa as opa
from workloads import adaptation, complex_gaussian, dpd_coeffs, pa_coeffs

from helpers import DPD_TOL, say

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _rel_per_branch(g, ref):
    return [float(np.linalg.norm(g[b] - ref[b]) / np.linalg.norm(ref[b])) for b in range(ref.shape[0])]


@pytest.mark.parametrize("with_ctrl,hist", [(False, "branch"), (True, "branch"), (True, "shared")])
def test_stateless_forward_matches_oracle(with_ctrl, hist):
    import torch
    from paper_1611_03226_amd import dfhip as D
    say(f"stateless forward ctrl={with_ctrl} {hist}")
    rng = np.random.default_rng(70)
    S, L, r, B, M = 3, 4096, 512, 10, 16
    x = complex_gaussian(rng, (S, L))
    h = dpd_coeffs(rng, B, M)
    ctrl = rng.integers(0, B + 1, (S, L // r)).astype(np.int32) if with_ctrl else None
    y = torch.empty((S, L), dtype=torch.complex64, device="cuda")
    D.df_dpd_forward(_t(x), None if ctrl is None else _t(ctrl), _t(h), y, r,
                     D.DF_HIST_SHARED if hist == "shared" else D.DF_HIST_BRANCH)
    torch.cuda.synchronize()
    ref = odpd.run_dpd_streams(x, ctrl, h, r if with_ctrl else L, hist)
    y = y.cpu().numpy()
    for s in range(S):
        num = np.linalg.norm((y[s] - ref[s]).reshape(-1, r), axis=1)
        den = np.linalg.norm(ref[s].reshape(-1, r), axis=1)
        assert (num[den > 0] / den[den > 0]).max() <= DPD_TOL
        assert (num[den == 0] == 0).all()


@pytest.mark.parametrize("B,M,r,with_ctrl", [(11, 16, 300, True), (13, 8, 96, True), (16, 16, 257, True),
                                              (16, 4, 64, True), (12, 8, 512, False), (16, 16, 1024, False)])
def test_stateless_forward_wide_branch_counts(B, M, r, with_ctrl):
    """n_branches_max 11..16 (the 16-branch instantiations of the tiled body
    and head pass) through the stateless call, against the oracle."""
    import torch
    from paper_1611_03226_amd import dfhip as D
    say(f"stateless forward B={B} M={M} r={r} ctrl={with_ctrl}")
    rng = np.random.default_rng(80 + B + M)
    S, nf = 2, 7
    L = nf * r
    x = complex_gaussian(rng, (S, L))
    h = dpd_coeffs(rng, B, M)
    ctrl = rng.integers(0, B + 1, (S, nf)).astype(np.int32) if with_ctrl else None
    y = torch.empty((S, L), dtype=torch.complex64, device="cuda")
    D.df_dpd_forward(_t(x), None if ctrl is None else _t(ctrl), _t(h), y, r)
    torch.cuda.synchronize()
    ref = odpd.run_dpd_streams(x, ctrl, h, r if with_ctrl else L, "branch")
    y = y.cpu().numpy()
    for s in range(S):
        num = np.linalg.norm((y[s] - ref[s]).reshape(-1, r), axis=1)
        den = np.linalg.norm(ref[s].reshape(-1, r), axis=1)
        assert (num[den > 0] / den[den > 0]).max() <= DPD_TOL
        assert (num[den == 0] == 0).all()


def test_mp_input_adjoint_matches_oracle():
    import torch
    from paper_1611_03226_amd import dfhip as D
    say("mp input adjoint")
    rng = np.random.default_rng(71)
    S, L = 4, 3000
    a = pa_coeffs(rng, 4, 4, sigma=0.2)
    u = complex_gaussian(rng, (S, L), rms=0.7)
    g = complex_gaussian(rng, (S, L))
    Gu = torch.empty((S, L), dtype=torch.complex64, device="cuda")
    D.df_mp_input_adjoint(_t(u), _t(a), _t(g), Gu)
    torch.cuda.synchronize()
    ref = opa.pa_input_vjp(u, a, g)
    got = Gu.cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    # element by element: FP32 rounding of each output relative to its own
    # magnitude, with an absolute floor at the RMS scale for near-zero outputs
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    elem = np.abs(got - ref) / (np.abs(ref) + 1e-3 * rms)
    print(f"mp input adjoint rel error {err:.3e}, worst element {elem.max():.3e}")
    assert err <= 1e-5
    assert elem.max() <= 1e-4


@pytest.mark.parametrize("with_ctrl,hist", [(False, "branch"), (True, "branch"), (True, "shared")])
def test_coefficient_adjoint_matches_fp64_adjoint(with_ctrl, hist):
    import torch
    from paper_1611_03226_amd import dfhip as D
    say(f"coeff adjoint ctrl={with_ctrl} {hist}")
    rng = np.random.default_rng(72)
    S, L, r, B, M = 3, 8192, 1024, 10, 16
    x = complex_gaussian(rng, (S, L))
    G = complex_gaussian(rng, (S, L))
    ctrl = rng.integers(0, B + 1, (S, L // r)).astype(np.int32) if with_ctrl else None
    grad = torch.empty((B, M), dtype=torch.complex64, device="cuda")
    work = torch.empty(D.df_dpd_coeff_adjoint_work_bytes(S, L, r, B, M), dtype=torch.uint8, device="cuda")
    hm = D.DF_HIST_SHARED if hist == "shared" else D.DF_HIST_BRANCH
    D.df_dpd_coeff_adjoint(_t(x), None if ctrl is None else _t(ctrl), _t(G), grad, r, work, hm)
    g1 = grad.cpu().numpy()
    D.df_dpd_coeff_adjoint(_t(x), None if ctrl is None else _t(ctrl), _t(G), grad, r, work, hm)
    g2 = grad.cpu().numpy()
    assert np.array_equal(g1.view(np.float32), g2.view(np.float32))      # deterministic
    ref = opa.dpd_coeff_vjp_streams(x, ctrl, G, B, M, r if with_ctrl else L, hist)
    rel = _rel_per_branch(g1, ref)
    print("per-branch rel error", ", ".join(f"{v:.1e}" for v in rel))
    assert max(rel) <= 1e-4


@pytest.mark.parametrize("B,M,r,with_ctrl", [(1, 4, 256, True), (5, 8, 512, True), (16, 16, 1024, True),
                                              (3, 5, 300, True), (7, 13, 2100, False), (16, 32, 640, True),
                                              (10, 16, 9000, True), (4, 7, 5000, True)])
def test_coefficient_adjoint_shapes(B, M, r, with_ctrl):
    """Branch and tap counts away from (10, 16): one branch, B_max 16, taps
    not a multiple of 4 (a partly used wavefront), ragged chunks, firings
    longer than a workgroup's 4096-sample span (pairs across span ends,
    branch histories); per branch against the FP64 adjoint."""
    import torch
    from paper_1611_03226_amd import dfhip as D
    say(f"coeff adjoint B={B} M={M} r={r} ctrl={with_ctrl}")
    rng = np.random.default_rng(90 + B * M)
    S, nf = 2, 5
    L = nf * r
    x = complex_gaussian(rng, (S, L))
    G = complex_gaussian(rng, (S, L))
    ctrl = rng.integers(0, B + 1, (S, nf)).astype(np.int32) if with_ctrl else None
    if with_ctrl:
        ctrl[0, 0] = B                            # every branch receives samples
    grad = torch.empty((B, M), dtype=torch.complex64, device="cuda")
    work = torch.empty(D.df_dpd_coeff_adjoint_work_bytes(S, L, r, B, M), dtype=torch.uint8, device="cuda")
    D.df_dpd_coeff_adjoint(_t(x), None if ctrl is None else _t(ctrl), _t(G), grad, r, work)
    ref = opa.dpd_coeff_vjp_streams(x, ctrl, G, B, M, r if with_ctrl else L, "branch")
    rel = _rel_per_branch(grad.cpu().numpy(), ref)
    print(f"B={B} M={M}: per-branch rel error max {max(rel):.1e}")
    assert max(rel) <= 1e-4


def test_autograd_gradient_matches_fp64_chain():
    import torch
    from paper_1611_03226_amd.autograd import adaptation_loss
    say("autograd vs fp64 adjoint chain")
    w = adaptation(seed=5, n_streams=4, length=8192)
    rng = np.random.default_rng(73)
    h0 = w.h0.astype(np.complex128) + 0.01 * (rng.standard_normal(w.h0.shape) + 1j * rng.standard_normal(w.h0.shape))
    h0 = h0.astype(np.complex64)
    x = _t(w.x)
    h = _t(h0).requires_grad_(True)
    a = _t(w.a)
    loss = adaptation_loss(x, h, a, 8192)
    loss.backward()
    L_ref, g_ref = opa.loss_grad(w.x, h0, w.a, 8192)
    assert abs(loss.item() - L_ref) <= 1e-4 * L_ref
    rel = _rel_per_branch(h.grad.cpu().numpy(), g_ref)
    print("autograd per-branch rel error", ", ".join(f"{v:.1e}" for v in rel))
    assert max(rel) <= 1e-4


def test_autograd_gradient_matches_finite_differences_of_gpu_forward():
    """Central differences (eps = 1e-3) of the GPU FP32 forward, loss summed in
    FP64; compared on the 32 largest gradient components."""
    import torch
    from paper_1611_03226_amd.autograd import DPDFunction, PAFunction, adaptation_loss
    say("autograd vs finite differences")
    w = adaptation(seed=5, n_streams=2, length=4096)
    x = _t(w.x)
    a = _t(w.a)
    h0 = torch.from_numpy(w.h0).to("cuda")
    h = h0.clone().requires_grad_(True)
    adaptation_loss(x, h, a, 4096).backward()
    g = h.grad.cpu().numpy()

    def loss64(hh):
        with torch.no_grad():
            v = PAFunction.apply(DPDFunction.apply(x, hh, 4096), a)
            e = (v - x).cpu().numpy().astype(np.complex128)
        return float(np.sum(e.real ** 2 + e.imag ** 2))

    flat = np.argsort(-np.abs(g).ravel())[:32]
    eps = 1e-3
    worst = 0.0
    for f in flat:
        b, m = divmod(int(f), g.shape[1])
        fd = 0j
        for unit in (1.0, 1j):
            hp = h0.clone()
            hm = h0.clone()
            hp[b, m] += eps * unit
            hm[b, m] -= eps * unit
            fd += (loss64(hp) - loss64(hm)) / (2 * eps) * unit
        worst = max(worst, abs(fd - g[b, m]) / abs(g[b, m]))
    print(f"FD vs adjoint, top-32 components: worst rel {worst:.2e}")
    assert worst <= 1e-2


def test_adaptation_loss_decreases():
    import torch
    from paper_1611_03226_amd.autograd import adaptation_loss
    say("adaptation loop")
    w = adaptation(seed=5, n_streams=8, length=16384)
    x = _t(w.x)
    a = _t(w.a)
    h = torch.from_numpy(w.h0).to("cuda").requires_grad_(True)
    opt = torch.optim.SGD([h], lr=5e-5)           # about 6.5 / samples; 1e-4 diverges (FP64 oracle)
    losses = []
    for _ in range(20):
        opt.zero_grad()
        loss = adaptation_loss(x, h, a, 16384)
        loss.backward()
        opt.step()
        losses.append(loss.item())
    print("loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.05 * losses[0]
    assert all(b <= a_ * 1.0001 for a_, b in zip(losses, losses[1:]))


def test_full_size_gradient_matches_fp64_adjoint():
    """64 streams x 65536 samples, 10 branches x 16 taps, at identity."""
    import torch
    from paper_1611_03226_amd.autograd import adaptation_loss
    say("adaptation full size gradient")
    w = adaptation()
    x = _t(w.x)
    a = _t(w.a)
    h = torch.from_numpy(w.h0).to("cuda").requires_grad_(True)
    loss = adaptation_loss(x, h, a, 65536)
    loss.backward()
    L_ref, g_ref = opa.loss_grad(w.x, w.h0, w.a, 65536)
    rel = _rel_per_branch(h.grad.cpu().numpy(), g_ref)
    print(f"full size: loss {loss.item():.6e} vs {L_ref:.6e}; per-branch rel", ", ".join(f"{v:.1e}" for v in rel))
    assert abs(loss.item() - L_ref) <= 1e-4 * L_ref
    assert max(rel) <= 1e-4
