"""Pins for the adaptation oracle (CPU only): the PA forward against the DPD
network it is a special case of, both adjoints against finite differences,
and the dot-product identity <J v, w> = <v, J* w> for the coefficient map."""
import numpy as np
import pytest

from oracle import dpd, pa
from workloads import adaptation, complex_gaussian, dpd_random, pa_coeffs


def _rdot(a, b):
    return float(np.real(np.sum(np.conj(a) * b)))


def test_pa_forward_is_an_all_active_dpd_network():
    rng = np.random.default_rng(0)
    a = pa_coeffs(rng)
    u = complex_gaussian(rng, 512, rms=0.5)
    v = pa.pa_forward(u, a)
    want = dpd.run_dpd(u, np.full(512 // 64, 4), a, 64)
    np.testing.assert_allclose(v, want, rtol=0, atol=1e-13)


def test_pa_input_vjp_matches_directional_finite_differences():
    rng = np.random.default_rng(1)
    a = pa_coeffs(rng, sigma=0.2)
    u = complex_gaussian(rng, 256, rms=0.6).astype(np.complex128)
    g = complex_gaussian(rng, 256).astype(np.complex128)
    G = pa.pa_input_vjp(u, a, g)
    for _ in range(4):
        du = complex_gaussian(rng, 256).astype(np.complex128)
        eps = 1e-6
        jdu = (pa.pa_forward(u + eps * du, a) - pa.pa_forward(u - eps * du, a)) / (2 * eps)
        lhs = _rdot(g, jdu)          # <g, J du>
        rhs = _rdot(G, du)           # <J* g, du>
        assert abs(lhs - rhs) <= 1e-7 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("hist", ["branch", "shared"])
def test_coefficient_vjp_dot_product_identity(hist):
    w = dpd_random(30, n_firings=10, r=16, n_branches_max=4, n_taps=6, n_delay=3, ctrl_low=0)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(w.h.shape) + 1j * rng.standard_normal(w.h.shape)
    wv = rng.standard_normal(10 * 16) + 1j * rng.standard_normal(10 * 16)
    Jv = dpd.run_dpd(w.x, w.ctrl, v, w.r, w.n_delay, hist=hist)     # the map is linear in h
    JTw = pa.dpd_coeff_vjp(w.x, w.ctrl, wv, 4, 6, w.r, w.n_delay, hist=hist)
    lhs, rhs = _rdot(Jv, wv), _rdot(v, JTw)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_loss_gradient_matches_central_finite_differences_all_params():
    """Reduced adaptation case: 2 streams x 512 samples, 4 branches x 4 taps."""
    w = adaptation(seed=5, n_streams=2, length=512, n_branches=4, n_taps=4)
    rng = np.random.default_rng(3)
    h = w.h0.astype(np.complex128) + 0.02 * (rng.standard_normal(w.h0.shape)
                                             + 1j * rng.standard_normal(w.h0.shape))
    L, grad = pa.loss_grad(w.x, h, w.a, 128)
    fd = pa.fd_grad(w.x, h, w.a, 128, eps=1e-3)
    assert L == pytest.approx(pa.loss(w.x, h, w.a, 128), rel=1e-12)
    for b in range(4):                           # per branch, so small high-order terms count
        rel = np.linalg.norm(grad[b] - fd[b]) / np.linalg.norm(fd[b])
        assert rel < 1e-5, (b, rel)


def test_loss_gradient_full_shape_sampled_params():
    """10 branches x 16 taps, a sample of coefficients from every branch."""
    w = adaptation(seed=5, n_streams=1, length=1024)
    h = w.h0.astype(np.complex128)
    L, grad = pa.loss_grad(w.x, h, w.a, 256)
    params = [(b, m) for b in range(10) for m in (0, 7, 15)]
    fd = pa.fd_grad(w.x, h, w.a, 256, eps=1e-3, params=params)
    for b, m in params:
        assert abs(grad[b, m] - fd[b, m]) <= 1e-5 * max(abs(fd[b, m]), 1e-12) + 1e-9, (b, m)
