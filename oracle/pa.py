"""Oracle for DPD coefficient adaptation.  TEST INFRASTRUCTURE ONLY.

The paper runs a fixed-coefficient DPD (Sec. 4.2) and gives no model for the
amplifier; adaptation is an extension of the method.  Readings:

* PA model: a memory polynomial v[n] = sum_k sum_q a[k][q] phi_k(u[n-q]),
  phi_k(z) = |z|^(2k) z (order 2k+1), zero input before the stream start.
* Loss L = sum_n |v[n] - x[n]|^2 with u = DPD_h(x) (all branches active).
* Gradients use the real-pair convention: for a complex quantity z the
  gradient is dL/dRe z + i dL/dIm z (the convention torch.autograd uses).
  With w = f(z), A = dw/dz and B = dw/dz* (Wirtinger), an upstream gradient
  g of w pulls back to g conj(A) + conj(g) B.

All arithmetic is complex128 / float64.
"""
from __future__ import annotations

import numpy as np

from .dpd import basis, read_stream, run_dpd, writes_branch


def phi(u: np.ndarray, k: int) -> np.ndarray:
    """phi_k(u) = (|u|^2)^k u, order 2k+1 (same odd basis as the DPD)."""
    return basis(u, k)


def pa_forward(u, a) -> np.ndarray:
    """v[n] = sum_k sum_q a[k][q] phi_k(u[n-q]) along the last axis."""
    u = np.asarray(u, np.complex128)
    a = np.asarray(a, np.complex128)
    K, Q = a.shape
    v = np.zeros_like(u)
    N = u.shape[-1]
    for k in range(K):
        f = phi(u, k)
        for q in range(Q):
            if q >= N:
                continue
            v[..., q:] += a[k, q] * f[..., :N - q]
    return v


def pa_input_vjp(u, a, g) -> np.ndarray:
    """G[n] = dL/dRe u[n] + i dL/dIm u[n] given g[n] = dL/dRe v[n] + i dL/dIm v[n].

    For order o = 2k+1: d phi/du = ((o+1)/2) |u|^(o-1) and
    d phi/du* = ((o-1)/2) |u|^(o-3) u^2, hence
    G[n] = sum_q [ g[n+q] conj(sum_k a[k][q] (k+1) p^k)
                   + conj(g[n+q]) sum_k a[k][q] k p^(k-1) u^2 ],  p = |u[n]|^2,
    where g beyond the stream end is zero and the k = 0 term of the second
    sum is absent (no negative power is formed)."""
    u = np.asarray(u, np.complex128)
    a = np.asarray(a, np.complex128)
    g = np.asarray(g, np.complex128)
    K, Q = a.shape
    N = u.shape[-1]
    p = u.real ** 2 + u.imag ** 2
    G = np.zeros_like(u)
    for q in range(Q):
        if q >= N:
            continue
        gs = np.zeros_like(g)
        gs[..., :N - q] = g[..., q:]                 # g[n+q]
        A = np.zeros_like(u)
        Bw = np.zeros_like(u)
        for k in range(K):
            A += a[k, q] * (k + 1) * p ** k
            if k >= 1:
                Bw += a[k, q] * k * p ** (k - 1) * u * u
        G += gs * np.conj(A) + np.conj(gs) * Bw
    return G


def dpd_coeff_vjp(x, ctrl, G, n_branches, n_taps, r, n_delay=0, initial=None,
                  hist="branch") -> np.ndarray:
    """grad_h[b][m] = sum_n G[n] conj(dy[n]/dh_b[m]).  y is linear and
    holomorphic in h, and dy[jr+i]/dh_b[m] is FIR_b's input sample at lag m,
    i.e. s_b^c[off_b(j) + i - m] (zero before the channel start) when b < B_j,
    else 0."""
    xs = read_stream(x, n_delay, initial)
    ctrl = np.asarray(ctrl)
    G = np.asarray(G, np.complex128)
    n = len(ctrl)
    grad = np.zeros((n_branches, n_taps), np.complex128)
    for b in range(n_branches):
        w = np.nonzero(writes_branch(ctrl, b, hist))[0]
        if len(w) == 0:
            continue
        sc = np.concatenate([basis(xs[j * r:(j + 1) * r], b) for j in w])
        rank = {int(j): k for k, j in enumerate(w)}
        for j in range(n):
            if ctrl[j] <= b:
                continue
            off = rank[j] * r
            g = G[j * r:(j + 1) * r]
            for m in range(n_taps):
                lo = off - m
                seg = np.zeros(r, np.complex128)
                src_lo = max(lo, 0)
                seg[src_lo - lo:] = sc[src_lo:lo + r]
                grad[b, m] += np.sum(g * np.conj(seg))
    return grad


def dpd_coeff_vjp_streams(x, ctrl, G, n_branches, n_taps, r, hist="branch") -> np.ndarray:
    """Sum of per-stream coefficient gradients (x, G: [S, L])."""
    x = np.asarray(x)
    grad = np.zeros((n_branches, n_taps), np.complex128)
    for s in range(x.shape[0]):
        c = np.full(x.shape[1] // r, n_branches) if ctrl is None else np.asarray(ctrl)[s]
        grad += dpd_coeff_vjp(x[s], c, G[s], n_branches, n_taps, r, hist=hist)
    return grad


def dpd_all_active(x, h, r) -> np.ndarray:
    """DPD output of every stream with all branches active in every firing."""
    x = np.asarray(x)
    h = np.asarray(h)
    S, L = x.shape
    return np.stack([run_dpd(x[s], np.full(L // r, h.shape[0]), h, r) for s in range(S)])


def loss(x, h, a, r) -> float:
    """L = sum |PA(DPD_h(x)) - x|^2 over all streams."""
    u = dpd_all_active(x, h, r)
    e = pa_forward(u, a) - np.asarray(x, np.complex128)
    return float(np.sum(e.real ** 2 + e.imag ** 2))


def loss_grad(x, h, a, r):
    """(L, dL/dh) by the adjoint chain: e = PA(u) - x, g = 2e,
    G = PA input VJP, grad_h = DPD coefficient VJP."""
    x = np.asarray(x)
    h = np.asarray(h, np.complex128)
    u = dpd_all_active(x, h, r)
    e = pa_forward(u, a) - x.astype(np.complex128)
    G = pa_input_vjp(u, a, 2.0 * e)
    grad = dpd_coeff_vjp_streams(x, None, G, h.shape[0], h.shape[1], r)
    return float(np.sum(e.real ** 2 + e.imag ** 2)), grad


def fd_grad(x, h, a, r, eps=1e-3, params=None) -> np.ndarray:
    """Central finite differences of ``loss`` on the real and imaginary part
    of every coefficient (or of the listed (b, m) pairs)."""
    h = np.asarray(h, np.complex128)
    grad = np.zeros_like(h)
    idx = params if params is not None else [(b, m) for b in range(h.shape[0]) for m in range(h.shape[1])]
    for b, m in idx:
        for unit in (1.0, 1j):
            hp = h.copy()
            hm = h.copy()
            hp[b, m] += eps * unit
            hm[b, m] -= eps * unit
            d = (loss(x, hp, a, r) - loss(x, hm, a, r)) / (2 * eps)
            grad[b, m] += d * unit
    return grad
