"""Tile autotuner for the persistent multi-instance predistortion launch.

Candidates are (tile_outputs, outputs_per_thread, blocks_per_cu) triples.
Each is timed on the GPU (HIP events around every HIP-graph replay of the
persistent chain, mean over the replays) over a subset of the instances, and
the fastest is cached in a JSON file keyed by device architecture, taps,
largest branch count, firing size and length class.

Cache file: $DFHIP_TUNE_CACHE, else ~/.cache/dfhip/tune.json.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

CANDIDATES = [(t, k, b) for t in (512, 1024, 2048) for k in (4, 8) for b in (2, 4, 8)
              if t % (64 * k) == 0 and t // k <= 512]


def cache_path() -> str:
    p = os.environ.get("DFHIP_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "dfhip", "tune.json")


def _key(arch, M, B_max, r, lengths) -> str:
    cls = int(round(math.log2(max(float(np.median(lengths)), 1.0))))
    return f"{arch}:M{M}:B{B_max}:r{r}:len2^{cls}"


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _pow2(n):
    p = 1
    while p < n:
        p <<= 1
    return p


def tune_instances(w, candidates=None, subset_stride: int = 4, reps: int = 4, force: bool = False, log=None):
    """Best (tile_outputs, outputs_per_thread, blocks_per_cu) for a workload of
    independent instances (workloads.InstancesWorkload)."""
    import torch
    from . import dfhip as D
    from .graph import Graph

    r, M = w.r, w.n_taps
    key = _key(_arch(), M, int(w.n_branches_max), r, w.lengths)
    cache = _load()
    if key in cache and not force:
        if log:
            log(f"tune: cached {key} -> {cache[key]['best']}")
        return tuple(cache[key]["best"])
    cands = candidates or [c for c in CANDIDATES if c[0] <= max(r, 64 * c[1])]
    sel = list(range(0, len(w.lengths), subset_stride))
    L = w.lengths[sel].astype(np.int64)
    nfs = (L // r).tolist()
    nb = len(cands) * (reps + 1)
    timings = {}
    with Graph(0) as G:
        chains = []
        for k, i in enumerate(sel):
            ch = G.dpd_chain(w.h[i], r, cap_x=_pow2(nb * int(L[k])), cap_ctrl=_pow2(nb * nfs[k]),
                             cap_y=_pow2(nb * int(L[k])))
            x_dev = torch.from_numpy(w.x[i]).cuda()
            c_dev = torch.from_numpy(w.ctrl(i)).cuda()
            for _ in range(nb):
                G.push(ch.x, x_dev)
                G.push(ch.ctrl, c_dev)
            chains.append(ch)
        actors = [c.actor for c in chains]
        for cand in cands:
            G.set_tile(*cand)
            G.fire_many(actors, nfs, persistent=True, graph=True)      # capture + warm
            G.sync()
            D.df_profile_enable(G.g, True)
            D.df_profile_read(G.g)
            for _ in range(reps):
                G.fire_many(actors, nfs, persistent=True, graph=True)
            G.sync()
            ms, n = D.df_profile_read(G.g)
            D.df_profile_enable(G.g, False)
            timings[cand] = ms * 1e-3 / max(n, 1)
            # drain outputs so the output rings never fill
            for ch, nf in zip(chains, nfs):
                y = torch.empty((reps + 1) * nf * r, dtype=torch.complex64, device="cuda")
                G.pop(ch.y, y)
    best = min(timings, key=timings.get)
    if log:
        log("tune: " + ", ".join(f"{c}:{t * 1e3:.3f}ms" for c, t in sorted(timings.items(), key=lambda kv: kv[1])))
    cache[key] = {"best": list(best), "ms": {str(list(c)): t * 1e3 for c, t in timings.items()}}
    _store(cache)
    return best
