"""torch.autograd functions over the HIP kernels, for DPD coefficient
adaptation through a fixed memory-polynomial PA model.

Gradients follow torch's convention for complex tensors, dL/dRe z + i dL/dIm z,
which is the convention of the library's adjoint kernels.

    u = DPDFunction.apply(x, h, r)        # predistortion, learnable h
    v = PAFunction.apply(u, a)            # fixed PA: v = sum a[k][q] |u|^(2k) u (delay q)
    loss = (v - x).abs().pow(2).sum()
    loss.backward()                        # h.grad from the hand-written adjoints

Every tensor here is complex64 on the GPU; all arithmetic of the forward and
backward passes runs in libdfhip.so on torch's current stream.
"""
from __future__ import annotations

import torch

from . import dfhip as D


def _stream():
    return torch.cuda.current_stream()


class DPDFunction(torch.autograd.Function):
    """y = DPD_h(x) for x [S, L], h [B, M]; ctrl [S, L/r] int32 or None (all
    branches active).  Backward: coefficient adjoint only (x is data)."""

    @staticmethod
    def forward(ctx, x, h, r: int, ctrl=None, hist: int = D.DF_HIST_BRANCH):
        x = x.contiguous()
        hc = h.detach().contiguous()
        y = torch.empty_like(x)
        D.df_dpd_forward(x, ctrl, hc, y, r, hist, stream=_stream())
        ctx.save_for_backward(x, ctrl if ctrl is not None else torch.empty(0))
        ctx.has_ctrl = ctrl is not None
        ctx.r, ctx.hist, ctx.hshape = r, hist, h.shape
        return y

    @staticmethod
    def backward(ctx, gy):
        x, ctrl = ctx.saved_tensors
        ctrl = ctrl if ctx.has_ctrl else None
        B, M = ctx.hshape
        S, L = x.shape
        grad_h = None
        if ctx.needs_input_grad[1]:
            grad_h = torch.empty((B, M), dtype=torch.complex64, device=x.device)
            nb = D.df_dpd_coeff_adjoint_work_bytes(S, L, ctx.r, B, M)
            work = torch.empty(max(nb, 8), dtype=torch.uint8, device=x.device)
            D.df_dpd_coeff_adjoint(x, ctrl, gy.contiguous(), grad_h, ctx.r, work, ctx.hist, stream=_stream())
        return None, grad_h, None, None, None


class PAFunction(torch.autograd.Function):
    """v = PA_a(u): memory polynomial with fixed coefficients a [K, Q]
    (orders 1, 3, .., 2K-1; delays 0..Q-1), evaluated by the predistortion
    kernel with all K branches active.  Backward: input adjoint."""

    @staticmethod
    def forward(ctx, u, a):
        u = u.contiguous()
        a = a.detach().contiguous()
        v = torch.empty_like(u)
        S, L = u.shape
        D.df_dpd_forward(u, None, a, v, L, D.DF_HIST_BRANCH, stream=_stream())
        ctx.save_for_backward(u, a)
        return v

    @staticmethod
    def backward(ctx, gv):
        u, a = ctx.saved_tensors
        gu = torch.empty_like(u)
        D.df_mp_input_adjoint(u, a, gv.contiguous(), gu, stream=_stream())
        return gu, None


def adaptation_loss(x, h, a, r):
    """L = sum |PA(DPD_h(x)) - x|^2."""
    u = DPDFunction.apply(x, h, r)
    v = PAFunction.apply(u, a)
    e = v - x
    return (e.real * e.real + e.imag * e.imag).sum()
