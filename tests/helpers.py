"""Shared helpers for the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np

# DPD FP32 vs FP64 tolerance: relative-to-RMS error per firing.
DPD_TOL = 1e-4


def say(msg: str) -> None:
    """Name the case before a GPU step (flushed, so a fault still shows it)."""
    print(f"[case] {msg}", file=sys.stderr, flush=True)


def rel_rms_per_firing(y, ref, r):
    """max_j ||y_j - ref_j|| / ||ref_j|| over firings with a non-zero reference,
    the global ratio, and the number of all-zero firings that are not exact."""
    y = np.asarray(y, np.complex128).reshape(-1, r)
    ref = np.asarray(ref, np.complex128).reshape(-1, r)
    num = np.linalg.norm(y - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    nz = den > 0
    worst = float((num[nz] / den[nz]).max()) if nz.any() else 0.0
    glob = float(np.linalg.norm(y - ref) / max(np.linalg.norm(ref), 1e-300))
    bad_zero = int(((~nz) & (num > 0)).sum())
    return worst, glob, bad_zero


def _pow2(n):
    p = 1
    while p < n:
        p <<= 1
    return p


def run_dpd_chain(G, w, hist="branch", batches=None, cap_x=0, cap_ctrl=0, cap_y=0):
    """Push a workload into a fresh DPD chain on graph G, fire it in the given
    batch sizes (default: one batch), pop all outputs.  Returns (y, chain)."""
    n = w.n_firings
    batches = batches or [n]
    assert sum(batches) == n
    big = max(batches) * w.r
    cap_x = cap_x or _pow2(n * w.r + w.n_delay)
    cap_y = cap_y or max(cap_x, _pow2(big))
    cap_ctrl = cap_ctrl or _pow2(n)
    ch = G.dpd_chain(w.h, w.r, w.n_delay, history=hist, cap_x=cap_x, cap_ctrl=cap_ctrl, cap_y=cap_y)
    out = []
    pos = 0
    xpos = 0
    for k in batches:
        # stream the inputs in as needed (exercises ring wrap with small capacities)
        need = (pos + k) * w.r - w.n_delay
        if need > xpos:
            G.push(ch.x, np.ascontiguousarray(w.x[xpos:need]))
            xpos = need
        G.push(ch.ctrl, np.ascontiguousarray(w.ctrl[pos:pos + k]))
        assert G.fire(ch.actor, k) == k
        buf = np.zeros(k * w.r, np.complex64)
        assert G.pop(ch.y, buf) == k * w.r
        out.append(buf)
        pos += k
    if xpos < len(w.x):
        G.push(ch.x, np.ascontiguousarray(w.x[xpos:]))
    return np.concatenate(out), ch
