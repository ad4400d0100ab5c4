#!/usr/bin/env python3
"""Throughput of the dynamic-rate actor hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]

One step = one batch of the predistortion actor at scale: 2**24 complex64
samples (OFDM-like input), 4096 firings of 4096 samples, per-firing control
tokens uniform in 1..10 active odd-order branches, 16-tap complex FIR per
branch.  Inputs (all W+K batches) are resident in the actor's HBM channels
before the timed region; a step is control intake + offset scan + actor
body + commit (one df_fire of 4096 firings).  The JSON line also carries,
as extras, motion detection (300 x 1920x1080 frames), the 64-firing chain
(batched vs per-firing), 1024 uneven instances (persistent HIP-graph launch
vs per-actor and per-firing launches) and one coefficient-adaptation step,
plus the oracle timed on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PER_FIRING = True
COPY = {"Bps": None}               # best measured HBM reference bandwidth (any access mix)
METRIC = "DPD Msamples/s + motion frames/s at 1 GPU; % HBM roofline; batched vs per-firing"
HBM_PEAK = 8.0e12                 # B/s, MI355X HBM3E
# MI355X's published FP32 vector peak (packed FP32: two FMAs per lane per
# cycle), the roofline's peak.  Every object here is compiled with packed
# FP32 disabled, so the issue ceiling of this code is half of it:
# 256 CUs x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz = 78.6 TFLOP/s.
FP32_PEAK = 157.3e12
VALU_PEAK = 256 * 4 * 16 * 2 * 2.4e9


# HBM traffic of the dominant kernel, from two rocprofv3 counter runs
# (FETCH_SIZE, WRITE_SIZE) scaled by the same counters on the stream-copy
# kernel; reported only while the kernel's sources are the ones profiled.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_dpd_tiled_dpd_scale_2p24_traffic.md")
KERNEL_SOURCES = ("paper_1611_03226_amd/csrc/k_dpd.hip", "paper_1611_03226_amd/csrc/dpd_tile.h",
                  "paper_1611_03226_amd/csrc/common.h")


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch recorded in the traffic summary, or None if it
    is missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(line.strip()[2:].split(": ", 1) for line in fh if line.startswith("- ") and ": " in line)
        if kv.get("source_sha256") != kernel_sources_sha256():
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def num(x, nd=4):
    """Rounded float, or None when not measured."""
    return None if x is None or x != x else round(x, nd)


def pow2(n):
    p = 1
    while p < n:
        p <<= 1
    return p


def dpd_flops(ctrl, r, M):
    """Algorithmic FLOPs of one batch, Horner form: per sample of a firing
    with B > 0 active branches, 3 (p = re^2 + im^2) + M * (4B + 4)."""
    B = np.asarray(ctrl, np.int64)
    return float(np.sum(np.where(B > 0, r * (3 + M * (4 * B + 4)), 0)))


# ----------------------------------------------------------------------- main line

def bench_dpd_scale(args, D, Graph, torch):
    global PER_FIRING
    PER_FIRING = not args.no_per_firing
    from workloads import dpd_scale
    w = dpd_scale()
    N, r, nf, M = len(w.x), w.r, w.n_firings, w.n_taps
    nb = args.warmup + args.steps
    G = Graph(0)
    ch = G.dpd_chain(w.h, r, cap_x=pow2(nb * N), cap_ctrl=pow2(nb * nf), cap_y=pow2(nb * N))
    x_dev = torch.from_numpy(w.x).cuda()
    c_dev = torch.from_numpy(w.ctrl).cuda()
    torch.cuda.synchronize()
    for _ in range(nb):
        G.push(ch.x, x_dev)
        G.push(ch.ctrl, c_dev)
    G.sync()
    for _ in range(args.warmup):
        G.fire(ch.actor, nf)
    G.sync()
    D.df_profile_enable(G.g, True)
    D.df_profile_read(G.g)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        G.fire(ch.actor, nf)
    G.sync()
    t1 = time.perf_counter()
    body_ms, n_body = D.df_profile_read(G.g)
    D.df_profile_enable(G.g, False)
    ms = (t1 - t0) * 1e3 / args.steps
    body = body_ms / max(n_body, 1)
    # the output of the last batch must be finite (parity at this size is a GPU test)
    y_dev = torch.empty(nb * N, dtype=torch.complex64, device="cuda")
    G.pop(ch.y, y_dev)
    G.sync()
    finite = bool(torch.isfinite(torch.view_as_real(y_dev[(nb - 1) * N:])).all().item())
    G.close()
    flops = dpd_flops(w.ctrl, r, M)
    res = dict(ms=ms, body_ms=body, flops=flops, bytes=16.0 * N, N=N, finite=finite,
               papr_db=w.notes["papr_db"], per_firing_ms=float("nan"))
    if not PER_FIRING:
        return res
    # per-firing launches on the same workload (one batch of 4096 df_fire(1))
    G = Graph(0)
    ch = G.dpd_chain(w.h, r, cap_x=pow2(2 * N), cap_ctrl=pow2(2 * nf), cap_y=pow2(2 * N))
    G.push(ch.x, x_dev)
    G.push(ch.ctrl, c_dev)
    G.push(ch.x, x_dev)
    G.push(ch.ctrl, c_dev)
    G.fire(ch.actor, nf)                     # warm
    G.sync()
    t0 = time.perf_counter()
    for _ in range(nf):
        G.fire(ch.actor, 1)
    G.sync()
    res["per_firing_ms"] = (time.perf_counter() - t0) * 1e3
    G.close()
    return res


# ----------------------------------------------------------------------- extras

def bench_chain(D, Graph, torch, reps=50):
    from workloads import dpd_chain
    w = dpd_chain()
    n, r = w.n_firings, w.r
    G = Graph(0)
    tot = 2 * reps + 2
    ch = G.dpd_chain(w.h, r, w.n_delay, cap_x=pow2(tot * n * r + 8), cap_ctrl=pow2(tot * n),
                     cap_y=pow2(tot * n * r))
    x_dev = torch.from_numpy(w.x).cuda()
    c_dev = torch.from_numpy(w.ctrl).cuda()
    torch.cuda.synchronize()
    for _ in range(tot):
        G.push(ch.x, x_dev)
        G.push(ch.ctrl, c_dev)
    G.fire(ch.actor, n)
    G.fire(ch.actor, n)
    G.sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        G.fire(ch.actor, n)
    G.sync()
    batched = (time.perf_counter() - t0) * 1e6 / reps
    per = float("nan")
    if PER_FIRING:
        t0 = time.perf_counter()
        for _ in range(reps):
            for _ in range(n):
                G.fire(ch.actor, 1)
        G.sync()
        per = (time.perf_counter() - t0) * 1e6 / reps
    G.close()
    return dict(workload="dpd chain 16384 samples, 64 firings of 256, B<=5, M=8, d=4",
                us_per_batch_batched=round(batched, 2), us_per_batch_per_firing=num(per, 2),
                speedup=num(per / batched, 2))


def bench_motion(D, Graph, torch, steps=3, warmup=1):
    from workloads import motion
    log("generating 300 frames of 1920x1080")
    m = motion()
    n, H, W = m.frames.shape
    nb = steps + warmup + 2
    G = Graph(0)
    mc = G.motion_chain(W, H, cap_in=pow2(nb * n), cap_out=pow2(nb * n))
    f_dev = torch.from_numpy(m.frames).cuda()
    torch.cuda.synchronize()
    for _ in range(nb):
        G.push(mc.cur, f_dev)
    for _ in range(warmup):
        G.fire(mc.actor, n)
    G.sync()
    e0 = G.status(mc.index)[1]
    D.df_profile_enable(G.g, True)
    D.df_profile_read(G.g)
    t0 = time.perf_counter()
    for _ in range(steps):
        G.fire(mc.actor, n)
    G.sync()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    body_ms, nl = D.df_profile_read(G.g)
    D.df_profile_enable(G.g, False)
    body = body_ms / max(nl, 1)
    emitted = (G.status(mc.index)[1] - e0) / steps
    per_ms = float("nan")
    if PER_FIRING:
        t0 = time.perf_counter()
        for _ in range(n):
            G.fire(mc.actor, 1)
        G.sync()
        per_ms = (time.perf_counter() - t0) * 1e3
    G.close()
    wh = W * H
    bytes_alg = n * wh + emitted * (wh + 8)
    return dict(workload="motion 300 frames 1920x1080 u8, threshold 25, 3x3 opening, emit at 0.1%",
                fps=round(n / (ms * 1e-3), 1), ms_per_batch=round(ms, 4), body_ms=round(body, 4),
                emit_fraction=round(emitted / n, 4),
                hbm_frac_alg=round(bytes_alg / (body * 1e-3) / HBM_PEAK, 4),
                achieved_GBps=round(bytes_alg / (body * 1e-3) / 1e9, 1),
                hbm_frac_of_best_reference=num(bytes_alg / (body * 1e-3) / COPY["Bps"]) if COPY["Bps"] else None,
                kernels={"bits": {"algorithmic_bytes": n * wh}, "expand": {"algorithmic_bytes": emitted * (wh + 8)}},
                per_frame_fps=num(n / (per_ms * 1e-3), 1), speedup_vs_per_frame=num(per_ms / ms, 2))


def bench_md_paper(D, Graph, torch, steps=5, warmup=2, n_frames=4096):
    """The paper's motion-detection pipeline (Sec. 4.1): Gauss 5x5 -> Thres ->
    Med 5-px on 320x240 u8 frames at token rate 4.  One step fires each actor
    n_frames/4 times, first as three actors over device FIFOs (three
    launches), then as one df_fire_pipeline call (one fused launch).  Inputs
    for every step are pushed before the timed regions."""
    from workloads import paper_motion
    rate, thr = 4, 20
    log(f"generating {n_frames} frames of 320x240")
    w = paper_motion(n_frames=n_frames)
    n, H, W = w.frames.shape
    nf = n // rate
    nb = 2 * (steps + warmup)
    G = Graph(0)
    p = G.paper_motion_pipeline(W, H, thr, rate, cap=pow2(n + 1), cap_io=pow2(nb * n + 1))
    f_dev = torch.from_numpy(w.frames).cuda()
    torch.cuda.synchronize()
    for _ in range(nb):
        G.push(p.inp, f_dev)
    wh = W * H

    def timed(fire):
        for _ in range(warmup):
            fire()
        G.sync()
        G.profile(True)
        G.profile_read()
        t0 = time.perf_counter()
        for _ in range(steps):
            fire()
        G.sync()
        return (time.perf_counter() - t0) * 1e3 / steps

    def kernel_entry(t_ms, byt):
        return {"ms": round(t_ms, 4), "algorithmic_bytes": byt, "GBps": round(byt / (t_ms * 1e-3) / 1e9, 1),
                "frac": round(byt / (t_ms * 1e-3) / HBM_PEAK, 4),
                "frac_of_best_reference": num(byt / (t_ms * 1e-3) / COPY["Bps"]) if COPY["Bps"] else None}

    ms_sep = timed(lambda: p.fire_all(G, nf))
    kern = {}
    for name, actor, frames_moved in (("gauss", p.gauss, 3), ("thres", p.thres, 3), ("med", p.med, 2)):
        t, nl = G.profile_read(actor)
        kern[name] = kernel_entry(t / max(nl, 1), frames_moved * n * wh)
    ms_fused = timed(lambda: p.fire_chain(G, nf))
    t, nl = G.profile_read(p.gauss)
    # fused launch: every input frame read, every output frame written, plus
    # the delay channel's token read and rewritten once per batch
    kern["fused"] = kernel_entry(t / max(nl, 1), 2 * n * wh + 2 * wh)
    G.profile(False)
    out = np.zeros((n, H, W), np.uint8)
    G.pop(p.out, out)
    nonempty = int((out.reshape(n, -1).max(axis=1) > 0).sum())
    # channel memory: the paper's Eq. (1) sizing at this rate vs this run's rings
    chans = [(p.inp, False), (p.g_cur, False), (p.g_delayed, True), (p.thr, False), (p.out, False)]
    eq1 = sum(D.df_paper_channel_bytes(wh, rate, d) for _, d in chans)
    rings = sum(G.status(f)[2] * wh for f, _ in chans)
    per_ms = float("nan")
    if PER_FIRING:
        # one more batch, fired one firing (4 frames) per actor call
        G.push(p.inp, f_dev)
        G.sync()
        t0 = time.perf_counter()
        for _ in range(nf):
            p.fire_all(G, 1)
        G.sync()
        per_ms = (time.perf_counter() - t0) * 1e3
    G.close()
    return dict(workload=f"paper motion detection: {n} frames 320x240 u8 per step, Gauss 5x5 -> Thres (T={thr}, "
                         "one-frame delay channel) -> Med 5-px, token rate 4",
                fps_three_actors=round(n / (ms_sep * 1e-3), 1), ms_per_batch_three_actors=round(ms_sep, 4),
                fps_fused=round(n / (ms_fused * 1e-3), 1), ms_per_batch_fused=round(ms_fused, 4),
                kernels=kern, frames_with_motion=nonempty,
                channel_bytes={"paper_eq1": eq1, "rings": rings,
                               "note": "Eq. (1) double/triple buffers hold one firing per channel; the rings "
                                       "hold whole batches (inner rings one batch, host-facing rings all "
                                       "batches pushed ahead of the timed steps)"},
                parity="tests/test_gpu_md_paper.py::test_full_size_sampled_frames and "
                       "::test_chain_full_size_sampled_frames (same workload and batch)",
                per_firing_fps=num(n / (per_ms * 1e-3), 1), speedup_vs_per_firing=num(per_ms / ms_sep, 2),
                paper_fps_context={"Carrizo A12-8800B + R7 (OpenCL 2.0)": 4614,
                                   "i7-4770 + Radeon HD 7750 (OpenCL 1.2)": 6063})


def bench_dpd_network(D, torch, steps=5, warmup=2):
    """The scale workload (2^24 samples, 4096 firings of 4096, B 1..10, M 16)
    through the network as the paper draws it (Poly -> per-branch channels ->
    FIR_b -> Adder, three kernels over the batch) against the fused actor
    body, both as stateless calls on the same device buffers."""
    from workloads import dpd_scale
    w = dpd_scale()
    N, r = len(w.x), w.r
    x = torch.from_numpy(w.x[None, :]).cuda()
    c = torch.from_numpy(w.ctrl[None, :]).cuda()
    h = torch.from_numpy(w.h).cuda()
    y = torch.empty_like(x)
    st = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(warmup):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_net = timed(lambda: D.df_dpd_forward_network(x, c, h, y, r, stream=st))
    ms_fused = timed(lambda: D.df_dpd_forward(x, c, h, y, r, D.DF_HIST_BRANCH, stream=st))
    eb = float(np.mean(w.ctrl))
    net_bytes = (4 * eb + 2) * N * 8            # P: read x, write E[B] channels; FIR: read+write; A: read, write y
    return dict(workload="dpd at scale as the P -> FIR_b -> A network with materialised branch channels",
                ms_network=round(ms_net, 4), ms_fused=round(ms_fused, 4),
                msps_network=round(N / (ms_net * 1e-3) / 1e6, 1), msps_fused=round(N / (ms_fused * 1e-3) / 1e6, 1),
                fused_speedup=round(ms_net / ms_fused, 2), network_algorithmic_bytes=net_bytes,
                network_GBps=round(net_bytes / (ms_net * 1e-3) / 1e9, 1),
                network_hbm_frac=round(net_bytes / (ms_net * 1e-3) / HBM_PEAK, 4),
                parity="tests/test_gpu_dpd_network.py::test_scale_workload_sampled_and_against_fused_body")


def bench_dpd_mask(D, Graph, torch, steps=40, warmup=10):
    """The scale workload (2^24 samples, 4096 firings of 4096, B_max 10,
    M 16) with bit-mask control tokens: each firing's token an arbitrary
    set of active branches, uniform over the 1023 non-empty sets (seeded).
    One step = one df_fire of the 4096 firings, inputs resident in HBM."""
    from workloads import dpd_scale
    w = dpd_scale()
    N, r, nf, M = len(w.x), w.r, w.n_firings, w.n_taps
    masks = np.random.default_rng(12).integers(1, 1 << 10, nf).astype(np.int32)
    nb = warmup + steps
    G = Graph(0)
    ch = G.dpd_chain(w.h, r, cap_x=pow2(nb * N), cap_ctrl=pow2(nb * nf), cap_y=pow2(nb * N), control="mask")
    x_dev = torch.from_numpy(w.x).cuda()
    c_dev = torch.from_numpy(masks).cuda()
    torch.cuda.synchronize()
    for _ in range(nb):
        G.push(ch.x, x_dev)
        G.push(ch.ctrl, c_dev)
    for _ in range(warmup):
        G.fire(ch.actor, nf)
    G.sync()
    D.df_profile_enable(G.g, True)
    D.df_profile_read(G.g)
    t0 = time.perf_counter()
    for _ in range(steps):
        G.fire(ch.actor, nf)
    G.sync()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    body_ms, nl = D.df_profile_read(G.g)
    G.close()
    body = body_ms / max(nl, 1)
    # work done: Horner over the highest active branch, zero terms included
    L = np.array([int(m).bit_length() for m in masks])
    flops = dpd_flops(L, r, M)
    return dict(workload="dpd at scale with bit-mask control tokens (arbitrary branch sets, uniform over the "
                         "1023 non-empty sets of 10 branches), 4096 firings of 4096, 16 taps",
                msps=round(N / (ms * 1e-3) / 1e6, 1), ms_per_step=round(ms, 4), body_ms=round(body, 4),
                mean_active_branches=round(float(np.mean([bin(int(m)).count("1") for m in masks])), 2),
                mean_horner_length=round(float(L.mean()), 2),
                body_fp32_frac=round(flops / (body * 1e-3) / FP32_PEAK, 4),
                parity="tests/test_gpu_dpd_mask.py (mask tokens through df_fire and df_fire_many)")


def bench_host_io(D, Graph, torch, steps=3, warmup=1):
    """PCIe-inclusive rates: each step pushes its batch from host memory,
    fires it, and pops the outputs back to host memory (the boundary's host
    pointer forms, which copy and synchronise).  DPD at scale (2^24 samples)
    and the paper's motion pipeline (4096 frames of 320x240, fused chain)."""
    from workloads import dpd_scale, paper_motion
    res = {}
    w = dpd_scale()
    N, nf = len(w.x), w.n_firings
    G = Graph(0)
    ch = G.dpd_chain(w.h, w.r, cap_x=pow2(2 * N), cap_ctrl=pow2(2 * nf), cap_y=pow2(2 * N))
    # page-locked host buffers (torch pin_memory) viewed as numpy arrays
    x = torch.from_numpy(np.ascontiguousarray(w.x)).pin_memory().numpy()
    c = torch.from_numpy(np.ascontiguousarray(w.ctrl)).pin_memory().numpy()
    y = torch.empty(N, dtype=torch.complex64).pin_memory().numpy()

    def dpd_step():
        G.push(ch.ctrl, c)
        G.push(ch.x, x)
        G.fire(ch.actor, nf)
        G.pop(ch.y, y)
    for _ in range(warmup):
        dpd_step()
    t0 = time.perf_counter()
    for _ in range(steps):
        dpd_step()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    G.close()
    res["dpd_scale"] = {"ms_per_step": round(ms, 3), "msps": round(N / (ms * 1e-3) / 1e6, 1),
                        "host_bytes_per_step": 16 * N + 4 * nf}
    # the same stream with input copies, firings and output copies overlapped
    # (df_stream_dpd, 8 batches of 512 firings, rings of two batches)
    nbat, fpb = 8, nf // 8
    G = Graph(0)
    ch = G.dpd_chain(w.h, w.r, cap_x=pow2(2 * fpb * w.r), cap_ctrl=pow2(2 * fpb), cap_y=pow2(2 * fpb * w.r))
    D.df_stream_dpd(G.g, ch.actor, x, c, y, nbat, fpb)          # warm-up
    t0 = time.perf_counter()
    for _ in range(steps):
        D.df_stream_dpd(G.g, ch.actor, x, c, y, nbat, fpb)
    ms = (time.perf_counter() - t0) * 1e3 / steps
    G.close()
    res["dpd_scale_overlapped"] = {"ms_per_step": round(ms, 3), "msps": round(N / (ms * 1e-3) / 1e6, 1),
                                   "batches": nbat, "firings_per_batch": fpb}
    m = paper_motion(n_frames=4096)
    n, H, W = m.frames.shape
    G = Graph(0)
    p = G.paper_motion_pipeline(W, H, 20, 4, cap=pow2(n + 1))
    f = torch.from_numpy(np.ascontiguousarray(m.frames)).pin_memory().numpy()
    out = torch.empty(f.shape, dtype=torch.uint8).pin_memory().numpy()

    def md_step():
        G.push(p.inp, f)
        p.fire_chain(G, n // 4)
        G.pop(p.out, out)
    for _ in range(warmup):
        md_step()
    t0 = time.perf_counter()
    for _ in range(steps):
        md_step()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    G.close()
    res["md_paper_fused"] = {"ms_per_step": round(ms, 3), "fps": round(n / (ms * 1e-3), 1),
                             "host_bytes_per_step": 2 * n * W * H}
    res["note"] = "host buffers page-locked; the HBM-resident rates are the main line and extras"
    return res


def bench_instances(D, Graph, torch, steps=2):
    from paper_1611_03226_amd import tune
    from workloads import dpd_instances
    w = dpd_instances()
    r, M = w.r, w.n_taps
    L = w.lengths.astype(np.int64)
    nfs = (L // r).tolist()
    tile = tune.tune_instances(w, log=log)
    modes = ("many", "persistent", "graph")
    nb = len(modes) * (steps + 1) + 1
    G = Graph(0)
    G.set_tile(*tile)
    xall = torch.from_numpy(np.concatenate(w.x)).cuda()
    offs = np.concatenate([[0], np.cumsum(L)])
    chains = []
    for i in range(len(L)):
        ch = G.dpd_chain(w.h[i], r, cap_x=pow2(nb * int(L[i])), cap_ctrl=pow2(nb * nfs[i]),
                         cap_y=pow2(nb * int(L[i])))
        c_dev = torch.from_numpy(w.ctrl(i)).cuda()
        for _ in range(nb):
            G.push(ch.x, xall[offs[i]:offs[i + 1]])
            G.push(ch.ctrl, c_dev)
        chains.append(ch)
    actors = [c.actor for c in chains]
    G.sync()
    res = {}
    for mode in modes:
        kw = dict(persistent=mode != "many", graph=mode == "graph")
        G.fire_many(actors, nfs, **kw)
        G.sync()
        D.df_profile_enable(G.g, True)
        D.df_profile_read(G.g)
        t0 = time.perf_counter()
        for _ in range(steps):
            G.fire_many(actors, nfs, **kw)
        G.sync()
        res[mode] = (time.perf_counter() - t0) * 1e3 / steps
        kms, kn = D.df_profile_read(G.g)
        D.df_profile_enable(G.g, False)
        res[mode + "_body_ms"] = kms / max(kn, 1) if mode != "many" else kms / steps
    res["per_firing"] = float("nan")
    if PER_FIRING:
        t0 = time.perf_counter()
        for a, nf in zip(actors, nfs):
            for _ in range(nf):
                G.fire(a, 1)
        G.sync()
        res["per_firing"] = (time.perf_counter() - t0) * 1e3
    G.close()
    total = float(L.sum())
    flops = sum(dpd_flops(np.full(nf, b), r, M) for nf, b in zip(nfs, w.n_branches))
    body = res["persistent_body_ms"]
    return dict(workload=f"1024 DPD instances, lognormal lengths 1024..262144 (sum {int(total)}), r=1024, "
                         f"B in 1..10 per instance, M=16",
                tile=dict(tile_outputs=tile[0], outputs_per_thread=tile[1], blocks_per_cu=tile[2]),
                msps_graph=round(total / (res["graph"] * 1e-3) / 1e6, 1),
                msps_persistent=round(total / (res["persistent"] * 1e-3) / 1e6, 1),
                msps_per_actor=round(total / (res["many"] * 1e-3) / 1e6, 1),
                msps_per_firing=num(total / (res["per_firing"] * 1e-3) / 1e6, 1),
                ms=dict((k, num(v)) for k, v in res.items()),
                persistent_fp32_frac=round(flops / (body * 1e-3) / FP32_PEAK, 4),
                persistent_frac_of_nonpacked_issue=round(flops / (body * 1e-3) / VALU_PEAK, 4),
                persistent_hbm_frac=round(16 * total / (body * 1e-3) / HBM_PEAK, 4),
                algorithmic_bytes=16 * total, algorithmic_flops=flops,
                speedup_graph_vs_per_firing=num(res["per_firing"] / res["graph"], 1))


def bench_adaptation(D, torch, steps=10, warmup=2):
    from paper_1611_03226_amd.autograd import adaptation_loss
    from workloads import adaptation
    w = adaptation()
    x = torch.from_numpy(w.x).cuda()
    a = torch.from_numpy(w.a).cuda()
    h = torch.from_numpy(w.h0).cuda().requires_grad_(True)
    S, L = w.x.shape
    opt = torch.optim.SGD([h], lr=6.5 / (S * L))
    losses = []

    def step():
        opt.zero_grad()
        loss = adaptation_loss(x, h, a, L)
        loss.backward()
        opt.step()
        return loss

    for _ in range(warmup):
        losses.append(step().item())
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        loss = step()
    ev1.record()
    torch.cuda.synchronize()
    step_ms = ev0.elapsed_time(ev1) / steps
    losses.append(loss.item())
    # the coefficient adjoint alone
    G = torch.randn(S, L, dtype=torch.complex64, device="cuda")
    grad = torch.empty_like(h)
    nb = D.df_dpd_coeff_adjoint_work_bytes(S, L, L, 10, 16)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    D.df_dpd_coeff_adjoint(x, None, G, grad, L, work, stream=torch.cuda.current_stream())
    ev0.record()
    for _ in range(steps):
        D.df_dpd_coeff_adjoint(x, None, G, grad, L, work, stream=torch.cuda.current_stream())
    ev1.record()
    torch.cuda.synchronize()
    adj_ms = ev0.elapsed_time(ev1) / steps
    adj_flops = S * L * 16 * (8 + 4 * 10)
    return dict(workload="adaptation 64 streams x 65536, DPD 10x16 learnable, PA orders 1..7 x 4 taps",
                step_ms=round(step_ms, 4), loss_first=losses[0], loss_after=losses[-1],
                coeff_adjoint_ms=round(adj_ms, 4),
                coeff_adjoint_fp32_frac=round(adj_flops / (adj_ms * 1e-3) / FP32_PEAK, 4),
                coeff_adjoint_frac_of_nonpacked_issue=round(adj_flops / (adj_ms * 1e-3) / VALU_PEAK, 4),
                coeff_adjoint_algorithmic_bytes=16 * S * L, coeff_adjoint_algorithmic_flops=adj_flops)


def hbm_reference(D, torch, nbytes, reps=10):
    """Achievable HBM bandwidth: the four reference access mixes over nbytes
    (bytes moved / time, HIP events on the launching stream); the best of
    them is the ceiling the actor kernels' fractions are taken against."""
    src = torch.ones(2 * nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    res = {"bytes": nbytes, "kernel": "k_hbm_ref<mode>"}
    moved = {D.HBM_REF_COPY: 2 * nbytes, D.HBM_REF_READ: nbytes, D.HBM_REF_WRITE: nbytes,
             D.HBM_REF_2R1W: 3 * nbytes}
    names = {D.HBM_REF_COPY: "copy", D.HBM_REF_READ: "read", D.HBM_REF_WRITE: "write",
             D.HBM_REF_2R1W: "two_reads_one_write"}
    best = 0.0
    for mode in (D.HBM_REF_COPY, D.HBM_REF_READ, D.HBM_REF_WRITE, D.HBM_REF_2R1W):
        D.df_hbm_ref(mode, src, dst, nbytes, stream=st)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            D.df_hbm_ref(mode, src, dst, nbytes, stream=st)
        ev1.record()
        torch.cuda.synchronize()
        bps = moved[mode] / (ev0.elapsed_time(ev1) * 1e-3 / reps)
        res[names[mode] + "_GBps"] = round(bps / 1e9, 1)
        best = max(best, bps)
    COPY["Bps"] = best
    res["best_GBps"] = round(best / 1e9, 1)
    res["best_frac_of_peak"] = round(best / HBM_PEAK, 4)
    del src, dst
    return res


def cpu_baseline(budget_s=12.0):
    """The oracle network on the same workload, pinned to one host core
    (the process's affinity is narrowed to one CPU for the timing, BLAS and
    OpenMP threads 1): a prefix of the batch sized to about budget_s, or
    whole batches repeated until budget_s has elapsed."""
    from oracle import dpd as odpd
    from workloads import dpd_scale
    w = dpd_scale()
    old_aff = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
    if old_aff:
        os.sched_setaffinity(0, {min(old_aff)})
    try:
        return _cpu_baseline(odpd, w, budget_s, old_aff)
    finally:
        if old_aff:
            os.sched_setaffinity(0, old_aff)


def _host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _cpu_baseline(odpd, w, budget_s, old_aff):
    r = w.r
    n = 16
    t0 = time.perf_counter()
    odpd.run_dpd(w.x[:n * r], w.ctrl[:n], w.h, r)
    dt = time.perf_counter() - t0
    n = int(min(w.n_firings, max(16, n * budget_s / max(dt, 1e-3))))
    reps, samples = 0, 0
    t0 = time.perf_counter()
    while True:
        odpd.run_dpd(w.x[:n * r], w.ctrl[:n], w.h, r)
        reps += 1
        samples += n * r
        dt = time.perf_counter() - t0
        if n < w.n_firings or dt >= budget_s:
            break
    what = (f"first {n} firings ({n * r} samples) of the 2^24-sample workload" if n < w.n_firings
            else f"the whole 2^24-sample batch (4096 firings), {reps} passes")
    return dict(value=round(samples / dt / 1e6, 4), unit="Msamples/s", cores=1, kind="oracle",
                sample=f"{what}, FP64 sequential dataflow scheduler, {dt:.1f} s",
                pinned_cpu=min(old_aff) if old_aff else None, cpu_model=_host_cpu_model(),
                host_nproc=os.cpu_count(), affinity_cpus=len(old_aff) if old_aff else None)


# ------------------------------------------------------------ counter summaries
#
# Each group: the profile file it writes, the bench legs its profiled runs
# need, and its kernels as (label, substring of the rocprofv3 kernel name,
# function of the bench JSON giving (algorithmic bytes, algorithmic FLOPs)
# per launch).  Counter runs are separate rocprofv3 passes over the same
# bench command: FETCH_SIZE, WRITE_SIZE, and the SQ pass below.

SQ_PASS = "SQ_INSTS_VALU SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_INSTS_VMEM_RD SQ_INSTS_LDS"
REF_COPY_KERNEL = "k_hbm_ref<0>"


def _md(b, k):
    return b["md_paper"]["kernels"][k]["algorithmic_bytes"], 0.0


COUNTER_GROUPS = {
    "dpd_scale": dict(
        file="k_dpd_tiled_dpd_scale_2p24_traffic.md", only="",
        title="k_dpd_tiled<16,4,10>, 2^24-sample workload (4096 firings of 4096, B 1..10, M 16)",
        kernels=[("body", "k_dpd_tiled<16, 4, 10, false>",
                  lambda b: (b["roofline"]["algorithmic_bytes_per_launch"],
                             b["roofline"]["algorithmic_flops_per_launch"]))]),
    "motion": dict(
        file="k_motion_bits_expand_motion_300x1080p_counters.md", only="motion",
        title="motion actor passes, 300 frames of 1920x1080 per launch (self-delay form)",
        kernels=[("bits", "k_motion_bits<4, true>", lambda b: (b["motion"]["kernels"]["bits"]["algorithmic_bytes"], 0.0)),
                 ("expand", "k_motion_expand<true>",
                  lambda b: (b["motion"]["kernels"]["expand"]["algorithmic_bytes"], 0.0))]),
    "instances": dict(
        file="k_pers_body_instances_1024_counters.md", only="instances",
        title="persistent body over the 1024-instance workload (26.7 M samples, r 1024, M 16)",
        kernels=[("body", "k_pers_body<16",
                  lambda b: (b["instances"]["algorithmic_bytes"], b["instances"]["algorithmic_flops"]))]),
    "adaptation": dict(
        file="k_adj_partial_adaptation_64x65536_counters.md", only="adaptation",
        title="coefficient adjoint, 64 streams x 65536 samples, 10 branches x 16 taps",
        kernels=[("coeff_adjoint", "k_adj_partial<10, 4>",
                  lambda b: (b["adaptation"]["coeff_adjoint_algorithmic_bytes"],
                             b["adaptation"]["coeff_adjoint_algorithmic_flops"]))]),
    "md_paper": dict(
        file="md_paper_pipeline_traffic.md", only="md_paper",
        title="paper motion-detection pipeline kernels, 4096 frames of 320x240 per launch",
        kernels=[("gauss", "k_gauss5_w<4, true, true>", lambda b: _md(b, "gauss")),
                 ("thres", "k_thres_v", lambda b: _md(b, "thres")),
                 ("med", "k_med5_w<4, true>", lambda b: _md(b, "med")),
                 ("fused", "k_mdp_fused<16>", lambda b: _md(b, "fused"))]),
}


def profile_command(group, label, counters):
    g = COUNTER_GROUPS[group]
    only = f"--only {g['only']} " if g["only"] else "--no-extras "
    regex = "|".join(sorted({k[1].split("<")[0] for k in g["kernels"]} | {"k_hbm_ref"}))
    return (f"rocprofv3 --pmc {counters} --kernel-include-regex '{regex}' -d pmc_{label} -o {label} "
            f"--output-format csv -- python3 /root/repo/bench.py --no-cpu {only}--no-per-firing --steps 3 "
            f"--warmup 1 > {label}.json")


def summarize_counters(group, bench_json, *csvs):
    """Counter summary of one kernel group from rocprofv3 --pmc CSVs (any
    passes) and the JSON line of the same bench command: per kernel the
    dispatches, mean duration under the profiler, HBM read and write bytes
    per launch (FETCH_SIZE / WRITE_SIZE divided by what the same counter
    reads per byte the copy reference moves), their ratio to the
    algorithmic bytes, and the SQ figures (VALU issue share: a wave64 VALU
    instruction occupies a 16-lane SIMD for 4 cycles; 1024 SIMDs at
    2.4 GHz)."""
    import csv
    g = COUNTER_GROUPS[group]
    with open(bench_json) as fh:
        b = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    labels = [("ref", REF_COPY_KERNEL)] + [(k[0], k[1]) for k in g["kernels"]]
    ctr, dur = {}, {}
    for path in csvs:
        with open(path) as fh:
            for row in csv.DictReader(fh):
                name = row["Kernel_Name"]
                key = next((lab for lab, pat in labels if pat in name), None)
                if key is None:
                    continue
                d = ctr.setdefault(key, {}).setdefault((path, row["Dispatch_Id"]), {})
                d[row["Counter_Name"]] = d.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
                dur.setdefault(key, {})[(path, row["Dispatch_Id"])] = \
                    (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-9

    def mean(key, counter):
        v = [d[counter] for d in ctr.get(key, {}).values() if counter in d]
        return (sum(v) / len(v), len(v)) if v else (None, 0)

    copy_bytes = b["hbm_ref"]["bytes"]
    fr = mean("ref", "FETCH_SIZE")[0] * 1024 / copy_bytes
    fw = mean("ref", "WRITE_SIZE")[0] * 1024 / copy_bytes
    lines = [f"# Counters: {g['title']}", "",
             "Commands (on the GPU host from the repository root, after `cd /tmp && export TMPDIR=/tmp`; "
             "each pass its own run):", ""]
    for lab, c in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE"), ("sq", SQ_PASS)):
        lines.append("    " + profile_command(group, lab, c))
    lines += ["    python3 /root/repo/bench.py --summarize-counters " + group +
              " fetch.json pmc_fetch/fetch_counter_collection.csv pmc_write/write_counter_collection.csv "
              "pmc_sq/sq_counter_collection.csv", "",
              f"Copy reference ({REF_COPY_KERNEL}, {copy_bytes} bytes read and written): FETCH_SIZE "
              f"{mean('ref', 'FETCH_SIZE')[0]:.1f} KiB, WRITE_SIZE {mean('ref', 'WRITE_SIZE')[0]:.1f} KiB per "
              f"dispatch; scale {fr:.4f} (read) and {fw:.4f} (write) counter bytes per byte moved.", "",
              "| kernel | dispatches | mean us (profiler) | HBM read B | HBM write B | algorithmic B | "
              "traffic / algorithmic | algorithmic GB/s | VALU issue share | waves | mean resident waves per CU |",
              "|---|---|---|---|---|---|---|---|---|---|---|"]
    kv = {}
    for lab, pat, fn in g["kernels"]:
        alg, flops = fn(b)
        f, nf = mean(lab, "FETCH_SIZE")
        w, nw = mean(lab, "WRITE_SIZE")
        rd = f * 1024 / fr if f is not None else None
        wr = w * 1024 / fw if w is not None else None
        ds = list(dur.get(lab, {}).values())
        t = sum(ds) / len(ds) if ds else None
        valu = mean(lab, "SQ_INSTS_VALU")[0]
        waves = mean(lab, "SQ_WAVES")[0]
        # per-dispatch ratios over the SQ pass's own durations
        sq = [(d, dur[lab][k]) for k, d in ctr.get(lab, {}).items() if "SQ_INSTS_VALU" in d and dur[lab][k] > 0]
        issue = (sum(d["SQ_INSTS_VALU"] * 4 / (1024 * 2.4e9 * t_) for d, t_ in sq) / len(sq)) if sq else None
        # SQ_WAVE_CYCLES: resident wave-cycles in units of 4 cycles, summed over the chip
        occ_l = [d["SQ_WAVE_CYCLES"] * 4 / (t_ * 2.4e9 * 256) for d, t_ in sq if "SQ_WAVE_CYCLES" in d]
        occ = sum(occ_l) / len(occ_l) if occ_l else None

        def fmt(v, f_="{:.0f}"):
            return "n/a" if v is None else f_.format(v)
        lines.append(f"| {pat} | {nf} / {nw} | {fmt(t * 1e6 if t else None, '{:.1f}')} | {fmt(rd)} | {fmt(wr)} | "
                     f"{alg:.0f} | {fmt((rd + wr) / alg if rd is not None and wr is not None else None, '{:.4f}')} | "
                     f"{fmt(alg / t / 1e9 if t else None, '{:.1f}')} | {fmt(issue, '{:.3f}')} | {fmt(waves)} | "
                     f"{fmt(occ, '{:.1f}')} |")
        kv[lab] = dict(rd=rd, wr=wr, alg=alg, flops=flops, t=t, valu=valu)
    lines.append("")
    for lab, pat, _ in g["kernels"]:
        d = kv[lab]
        if d["rd"] is not None and d["wr"] is not None:
            lines.append(f"- {lab}.hbm_bytes_per_launch: {d['rd'] + d['wr']:.0f}")
        lines.append(f"- {lab}.algorithmic_bytes_per_launch: {d['alg']:.0f}")
        if d["flops"]:
            lines.append(f"- {lab}.algorithmic_flops_per_launch: {d['flops']:.0f}")
    if group == "dpd_scale":
        d = kv["body"]
        if d["rd"] is not None and d["wr"] is not None:
            lines.append(f"- hbm_bytes_per_launch: {d['rd'] + d['wr']:.0f}")
        lines.append(f"- source_sha256: {b['roofline']['kernel_sources_sha256']}")
    lines.append("")
    out = os.path.join(ROOT, "profiles", g["file"])
    with open(out, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


STATS_RUNS = {
    # file, title, bench arguments of the traced run
    "dpd_scale": ("k_dpd_tiled_dpd_scale_2p24_kernel_stats.md",
                  "predistortion actor at scale (2^24 samples, 4096 firings of 4096, B 1..10, M 16), "
                  "20 timed + 3 warm-up batches",
                  "--no-cpu --no-extras --no-per-firing --steps 20 --warmup 3"),
    "extras": ("motion_instances_adaptation_kernel_stats.md",
               "motion (300 x 1920x1080), mask tokens at scale, 1024 lognormal DPD instances (persistent / "
               "graph / per-actor), adaptation step; plus the main line at 3 batches",
               "--no-cpu --no-per-firing --only motion,dpd_mask,instances,adaptation --steps 3 --warmup 1"),
    "dpd_network": ("dpd_network_scale_kernel_stats.md",
                    "predistortion at scale (2^24 samples, 4096 firings of 4096, B 1..10, M 16) as the Poly -> "
                    "FIR_b -> Adder network with materialised branch channels, beside the fused stateless body",
                    "--no-cpu --no-per-firing --only dpd_network --steps 5 --warmup 2"),
    "md_paper": ("md_paper_pipeline_kernel_stats.md",
                 "paper motion-detection pipeline, 4096 frames of 320x240 per step (three actors and fused), "
                 "5 timed + 2 warm-up steps; plus the main line",
                 "--no-cpu --no-per-firing --only md_paper --steps 5 --warmup 2"),
}


def stats_command(run):
    return (f"rocprofv3 --kernel-trace --stats -d kt_{run} -o kt_{run} --output-format csv -- python3 "
            f"/root/repo/bench.py {STATS_RUNS[run][2]} > kt_{run}.json")


def summarize_kernel_stats(run, stats_csv):
    """profiles/ summary of a rocprofv3 --kernel-trace --stats run (the
    kernel_stats.csv it writes): per kernel the calls and durations."""
    import csv
    fname, title, _ = STATS_RUNS[run]
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# Kernel trace: {title}", "",
             "Command (on the GPU host, after `cd /tmp && export TMPDIR=/tmp`):", "",
             "    " + stats_command(run),
             f"    python3 /root/repo/bench.py --summarize-kernel-stats {run} kt_{run}/kt_{run}_kernel_stats.csv", "",
             "rocprofv3 kernel statistics (durations in microseconds):", "",
             "| kernel | calls | total us | average us | min us | max us | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows[:24]:
        name = r["Name"][:110]
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    lines.append("")
    with open(os.path.join(ROOT, "profiles", fname), "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--only", default="", help="comma list of extras to run: chain,motion,md_paper,dpd_network,dpd_mask,host_io,instances,"
                         "adaptation")
    ap.add_argument("--no-per-firing", action="store_true", help="skip the per-firing launch comparisons")
    ap.add_argument("--calibrate-copy", type=int, default=1024, metavar="MIB",
                    help="stream-copy reference size in MiB (bandwidth and traffic-counter reference; 0: off)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="ARG",
                    help="GROUP BENCH_JSON CSV...: write profiles/ counter summary of a kernel group "
                         f"({', '.join(COUNTER_GROUPS)}) from rocprofv3 --pmc runs of this script (no GPU)")
    ap.add_argument("--print-profile-commands", metavar="GROUP",
                    help="print the rocprofv3 commands of a counter group's passes")
    ap.add_argument("--summarize-kernel-stats", nargs=2, metavar=("RUN", "STATS_CSV"),
                    help=f"write the profiles/ kernel-trace summary of a traced run ({', '.join(STATS_RUNS)})")
    ap.add_argument("--print-stats-command", metavar="RUN", help="print the rocprofv3 kernel-trace command of a run")
    args = ap.parse_args()
    if args.summarize_counters:
        if len(args.summarize_counters) < 3 or args.summarize_counters[0] not in COUNTER_GROUPS:
            ap.error("--summarize-counters takes GROUP BENCH_JSON CSV...")
        summarize_counters(*args.summarize_counters)
        return
    if args.summarize_kernel_stats:
        summarize_kernel_stats(*args.summarize_kernel_stats)
        return
    if args.print_stats_command:
        print(stats_command(args.print_stats_command))
        return
    if args.print_profile_commands:
        for lab, c in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE"), ("sq", SQ_PASS)):
            print(profile_command(args.print_profile_commands, lab, c))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this build runs on one "
              f"MI355X; sharding across GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1611_03226_amd import dfhip as D
    from paper_1611_03226_amd.graph import Graph
    torch.cuda.set_device(0)

    log("dpd at scale")
    m = bench_dpd_scale(args, D, Graph, torch)
    value = m["N"] / (m["ms"] * 1e-3) / 1e6
    body_s = m["body_ms"] * 1e-3
    achieved = m["flops"] / body_s / 1e12
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "Msamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(m["ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dpd at scale: 2^24 complex64 OFDM-like samples, 4096 firings of 4096, "
                               "control uniform 1..10 branches (odd orders to 19), 16 taps",
                   "n_samples": m["N"], "firing_size": 4096, "n_branches_max": 10, "n_taps": 16},
        "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": round(FP32_PEAK / 1e12, 1),
                     "unit": "TFLOP/s", "frac": round(achieved * 1e12 / FP32_PEAK, 4), "traffic": measured_traffic(),
                     "algorithmic_bytes_per_launch": m["bytes"], "kernel_sources_sha256": kernel_sources_sha256(),
                     "kernel": "k_dpd_tiled<16,4,10>", "kernel_ms": round(m["body_ms"], 4),
                     "algorithmic_flops_per_launch": m["flops"],
                     "frac_of_nonpacked_issue": round(achieved * 1e12 / VALU_PEAK, 4),
                     "hbm_frac": round(m["bytes"] / body_s / HBM_PEAK, 4)},
        "per_firing": {"ms_per_batch": num(m["per_firing_ms"], 3),
                       "msps": num(m["N"] / (m["per_firing_ms"] * 1e-3) / 1e6, 1),
                       "batched_speedup": num(m["per_firing_ms"] / m["ms"], 1)},
        "outputs_finite": m["finite"],
        "parity": "tests/test_gpu_dpd.py::test_scale_workload_full_size (same workload and launch shape, "
                  "every firing against the oracle)",
    }
    if args.calibrate_copy:
        out["hbm_ref"] = hbm_reference(D, torch, args.calibrate_copy << 20)
        out["roofline"]["hbm_frac_of_best_reference"] = round(m["bytes"] / body_s / COPY["Bps"], 4)
    only = set(filter(None, args.only.split(",")))
    extras = [("chain", lambda: bench_chain(D, Graph, torch)),
              ("motion", lambda: bench_motion(D, Graph, torch)),
              ("md_paper", lambda: bench_md_paper(D, Graph, torch)),
              ("dpd_network", lambda: bench_dpd_network(D, torch)),
              ("dpd_mask", lambda: bench_dpd_mask(D, Graph, torch)),
              ("host_io", lambda: bench_host_io(D, Graph, torch)),
              ("instances", lambda: bench_instances(D, Graph, torch)),
              ("adaptation", lambda: bench_adaptation(D, torch))]
    if not args.no_extras:
        for name, fn in extras:
            if only and name not in only:
                continue
            log(name)
            out[name] = fn()
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
