"""Oracle for the dynamic predistortion (DPD) network.  TEST INFRASTRUCTURE ONLY.

Sec. 4.2 describes the application: a configuration actor C reconfigures the
Poly actor P and the Adder actor A at run time so that a chosen set of
parallel FIR filters processes the input; complex samples travel as float
pairs.  The paper gives neither the polynomial nor the branch selection rule;
this oracle takes these readings:

* P computes, for branch b, the odd-order basis psi_b(x) = |x|^(2b) x
  (order 2b+1), formed as (re^2 + im^2)^b * x without a square root.
* A control token B selects the prefix of branches b < B (B = 0: none).
* One token = one complex sample; a firing moves r samples.
* FIR_b is a static actor; its delay line only advances on tokens it
  consumes, so after an inactive stretch its history is the tail of its own
  last active firing ("branch" history, the literal dataflow semantics of
  Sec. 2.2).  The alternative "shared" history keeps every FIR fed on every
  firing (P always produces all branches, A still sums b < B).
* FIR state starts at zero; delay tokens on the input channel are zeros
  unless given.

Everything is complex128 / float64.
"""
from __future__ import annotations

import numpy as np

from .dataflow import Actor, Fifo, Scheduler, Sink, Source


def basis(x: np.ndarray, b: int) -> np.ndarray:
    """psi_b(x) = (|x|^2)^b x, the order-(2b+1) odd basis function."""
    x = np.asarray(x, np.complex128)
    p = x.real * x.real + x.imag * x.imag
    return p ** b * x


def _check_ctrl(B, n_branches_max, control="count"):
    B = int(B)
    if control == "mask":
        if B < 0 or B >= (1 << n_branches_max):
            raise ValueError(f"control mask {B} outside 0..2^{n_branches_max}-1")
        return B
    if B < 0 or B > n_branches_max:
        raise ValueError(f"control token {B} outside 0..{n_branches_max}")
    return B


def active(token, b, control="count") -> bool:
    """Whether branch b is active in a firing: "count" tokens activate the
    prefix b < B (the reading of Sec. 4.2 used throughout); "mask" tokens
    activate the set bits, any subset of the branches (the paper's "which
    set of the FIR filters")."""
    token = int(token)
    return bool((token >> b) & 1) if control == "mask" else b < token


class Poly(Actor):
    """P: dynamic actor.  Control token B fixes the rate of output s_b to r
    for b < B and to 0 otherwise ("branch" history); with ``shared`` every
    output keeps rate r.  Input x always has rate r."""

    def __init__(self, name, n_branches_max, shared=False, control="count"):
        super().__init__(name)
        self.B_max = n_branches_max
        self.shared = shared
        self.mode = control

    def control(self, token):
        B = _check_ctrl(token, self.B_max, self.mode)
        rin = {"x": self.inputs["x"].rate}
        rout = {}
        for b in range(self.B_max):
            f = self.outputs[f"s{b}"]
            rout[f"s{b}"] = f.rate if (self.shared or active(B, b, self.mode)) else 0
        return rin, rout

    def fire(self, consumed, token):
        x = consumed["x"]
        return {f"s{b}": basis(x, b) for b in range(self.B_max)
                if self.shared or active(token, b, self.mode)}


class FIR(Actor):
    """FIR_b: static actor, rate r in and out.  u[t] = sum_m h[m] s[t-m] with
    the delay line holding the last M-1 consumed inputs (zeros initially)."""

    def __init__(self, name, taps, initial_state=None):
        super().__init__(name)
        self.h = np.asarray(taps, np.complex128)
        M = len(self.h)
        self.state = np.zeros(M - 1, np.complex128) if initial_state is None \
            else np.asarray(initial_state, np.complex128).copy()

    def fire(self, consumed, token):
        s = consumed["in"]
        M = len(self.h)
        ext = np.concatenate([self.state, s])          # ext[M-1+t] = s[t]
        n = len(s)
        u = np.zeros(n, np.complex128)
        for m in range(M):
            u += self.h[m] * ext[M - 1 - m: M - 1 - m + n]
        self.state = ext[len(ext) - (M - 1):] if M > 1 else self.state
        return {"out": u}


class Adder(Actor):
    """A: dynamic actor.  Control token B fixes input u_b's rate to r for b < B
    and 0 otherwise ("branch" history; with ``shared`` every u_b keeps rate r
    but only b < B is summed).  Output y always has rate r; y = sum_{b<B} u_b,
    zero when B = 0."""

    def __init__(self, name, n_branches_max, shared=False, control="count"):
        super().__init__(name)
        self.B_max = n_branches_max
        self.shared = shared
        self.mode = control

    def control(self, token):
        B = _check_ctrl(token, self.B_max, self.mode)
        rin = {}
        for b in range(self.B_max):
            f = self.inputs[f"u{b}"]
            rin[f"u{b}"] = f.rate if (self.shared or active(B, b, self.mode)) else 0
        return rin, {"y": self.outputs["y"].rate}

    def fire(self, consumed, token):
        r = self.outputs["y"].rate
        y = np.zeros(r, np.complex128)
        for b in range(self.B_max):
            if active(token, b, self.mode):
                y = y + consumed[f"u{b}"]
        return {"y": y}


class DPDNetwork:
    """SrcX -> [x: rate r, d initial tokens] -> P -> s_b -> FIR_b -> u_b -> A -> y -> SinkY,
    with SrcC writing every control token to both cP and cA (control fan-out
    of the configuration actor C)."""

    def __init__(self, x, ctrl, h, r, n_delay=0, initial=None, hist="branch", control="count"):
        h = np.asarray(h, np.complex128)
        B_max, M = h.shape
        if hist not in ("branch", "shared"):
            raise ValueError(hist)
        shared = hist == "shared"
        self.r = r
        if initial is None:
            initial = np.zeros(n_delay, np.complex128)
        self.fx = Fifo("x", dtype=np.complex128, rate=r, initial=np.asarray(initial, np.complex128))
        self.fcP = Fifo("cP", dtype=np.int64, rate=1)
        self.fcA = Fifo("cA", dtype=np.int64, rate=1)
        self.fs = [Fifo(f"s{b}", dtype=np.complex128, rate=r) for b in range(B_max)]
        self.fu = [Fifo(f"u{b}", dtype=np.complex128, rate=r) for b in range(B_max)]
        self.fy = Fifo("y", dtype=np.complex128, rate=r)
        ctrl = np.asarray(ctrl, np.int64)
        self.srcx = Source("SrcX", {"x": np.asarray(x, np.complex128)})
        self.srcx.connect_out("x", self.fx)
        self.srcc = Source("SrcC", {"cP": ctrl, "cA": ctrl})
        self.srcc.connect_out("cP", self.fcP)
        self.srcc.connect_out("cA", self.fcA)
        self.P = Poly("P", B_max, shared, control)
        self.P.connect_ctrl(self.fcP)
        self.P.connect_in("x", self.fx)
        self.firs = []
        for b in range(B_max):
            self.P.connect_out(f"s{b}", self.fs[b])
            f = FIR(f"FIR{b}", h[b])
            f.connect_in("in", self.fs[b])
            f.connect_out("out", self.fu[b])
            self.firs.append(f)
        self.A = Adder("A", B_max, shared, control)
        self.A.connect_ctrl(self.fcA)
        for b in range(B_max):
            self.A.connect_in(f"u{b}", self.fu[b])
        self.A.connect_out("y", self.fy)
        self.sink = Sink("SinkY")
        self.sink.connect_in("y", self.fy)
        self.sched = Scheduler([self.srcx, self.srcc, self.P, *self.firs, self.A, self.sink])

    def run(self, policy="round_robin", seed=0) -> np.ndarray:
        self.sched.run(policy=policy, seed=seed)
        return self.sink.collected("y")


def run_dpd(x, ctrl, h, r, n_delay=0, initial=None, hist="branch",
            policy="round_robin", seed=0, control="count") -> np.ndarray:
    """Output stream y (complex128) of the DPD network fired to quiescence."""
    return DPDNetwork(x, ctrl, h, r, n_delay, initial, hist, control).run(policy, seed)


def run_dpd_streams(x, ctrl, h, r, hist="branch", control="count") -> np.ndarray:
    """Independent networks, one per row of x [S, L] (zero initial state, no
    delay tokens); ctrl [S, L/r] or None for all branches active."""
    x = np.asarray(x)
    h = np.asarray(h)
    S, L = x.shape
    out = np.zeros((S, L), np.complex128)
    for s in range(S):
        c = np.full(L // r, h.shape[0]) if ctrl is None else np.asarray(ctrl)[s]
        out[s] = run_dpd(x[s], c, h, r, hist=hist, control=control)
    return out


# ------------------------------------------------------------- rate / offset tables

def writes_branch(ctrl, b, hist="branch", control="count") -> np.ndarray:
    """Firings that write channel s_b: those in which branch b is active
    ("branch"), every firing ("shared")."""
    ctrl = np.asarray(ctrl)
    if hist == "shared":
        return np.ones(len(ctrl), bool)
    return np.array([active(c, b, control) for c in ctrl], bool)


def firing_tables(ctrl, n_branches_max, r, hist="branch", control="count"):
    """Per-firing tables implied by the firing rule (Sec. 2.2), by plain loops:

    rates[b][j]   token rate of A's input port u_b in firing j: r if branch b
                  is active in firing j (b < B_j for count tokens, bit b set
                  for mask tokens), else 0
    offsets[b][j] token offset of firing j's block on channel s_b: r times the
                  number of earlier firings that wrote s_b
    prev[b][j]    last earlier firing that wrote s_b (-1: none); its tail is
                  FIR_b's history at the start of firing j
    last[b]       last firing of the batch that wrote s_b (-1: none)
    """
    n = len(ctrl)
    rates = np.zeros((n_branches_max, n), np.int64)
    offsets = np.zeros((n_branches_max, n), np.int64)
    prev = np.full((n_branches_max, n), -1, np.int64)
    last = np.full(n_branches_max, -1, np.int64)
    for b in range(n_branches_max):
        written = 0
        lastw = -1
        for j in range(n):
            B = _check_ctrl(ctrl[j], n_branches_max, control)
            on = active(B, b, control)
            rates[b, j] = r if on else 0
            offsets[b, j] = r * written
            prev[b, j] = lastw
            if hist == "shared" or on:
                written += 1
                lastw = j
        last[b] = lastw
    return rates, offsets, prev, last


# ------------------------------------------------------------- independent closed forms

def read_stream(x, n_delay=0, initial=None) -> np.ndarray:
    """Tokens as the reader of the x channel sees them: initial tokens first."""
    init = np.zeros(n_delay, np.complex128) if initial is None else np.asarray(initial, np.complex128)
    return np.concatenate([init, np.asarray(x, np.complex128)])


def compacted_closed_form(x, ctrl, h, r, n_delay=0, initial=None, hist="branch") -> np.ndarray:
    """Second formulation used to cross-check the network: s_b^c is the
    concatenation of psi_b(window_j) over the firings that write s_b, FIR_b
    is one causal convolution over s_b^c with zero initial state, and
    y_j[t] = sum_{b<B_j} (h_b * s_b^c)[off_b(j) + t]."""
    h = np.asarray(h, np.complex128)
    B_max, M = h.shape
    xs = read_stream(x, n_delay, initial)
    ctrl = np.asarray(ctrl)
    n = min(len(ctrl), len(xs) // r)
    ctrl = ctrl[:n]
    y = np.zeros(n * r, np.complex128)
    for b in range(B_max):
        w = np.nonzero(writes_branch(ctrl, b, hist))[0]
        if len(w) == 0:
            continue
        sc = np.concatenate([basis(xs[j * r:(j + 1) * r], b) for j in w])
        u = np.convolve(h[b], sc)[:len(sc)]
        for k, j in enumerate(w):
            if ctrl[j] > b:
                y[j * r:(j + 1) * r] += u[k * r:(k + 1) * r]
    return y


def output_at(xs, ctrl, h, r, idx, hist="branch") -> np.ndarray:
    """y at the given output positions, one by one, from the definition:
    y[jr+i] = sum_{b<B_j} sum_m h_b[m] * s_b^c[off_b(j) + i - m], where the
    channel position is mapped back to the firing that wrote it.  ``xs`` is
    the read stream (delay tokens included).  Used for sampled checks of
    large runs."""
    h = np.asarray(h, np.complex128)
    B_max, M = h.shape
    ctrl = np.asarray(ctrl)
    writers = [np.nonzero(writes_branch(ctrl, b, hist))[0] for b in range(B_max)]
    ranks = []
    for b in range(B_max):
        rk = np.full(len(ctrl), -1, np.int64)
        rk[writers[b]] = np.arange(len(writers[b]))
        ranks.append(rk)
    out = np.zeros(len(idx), np.complex128)
    for k, t in enumerate(np.asarray(idx)):
        j, i = divmod(int(t), r)
        acc = 0j
        for b in range(int(ctrl[j])):
            pos0 = ranks[b][j] * r + i           # this firing writes s_b, rank known
            for m in range(M):
                pos = pos0 - m
                if pos < 0:
                    continue
                wj = writers[b][pos // r]
                acc += h[b, m] * basis(xs[wj * r + pos % r], b)
        out[k] = acc
    return out
