"""Oracle for the paper's motion-detection pipeline.  TEST INFRASTRUCTURE ONLY.

Sec. 4.1: five actors Src -> Gauss -> Thres -> Med -> Sink on 8-bit
grayscale frames (one frame per token).  Gauss is a 5x5 Gaussian filter that
leaves the two top and the two bottom pixel rows unfiltered; Thres subtracts
consecutive frames and thresholds against a fixed constant; Med is a
5-pixel median filter.  Two channels join Gauss to Thres; one of them holds
one initial token, the one-frame delay that lets Thres see the previous
filtered frame.  On the GPU every channel has token rate 4 (Sec. 4.1).

The paper leaves several details open; this module fixes them so:
  * Gauss weights: the 5x5 binomial kernel, outer product of (1,4,6,4,1)
    with itself, sum 256; the weighted sum S of a pixel's neighbourhood is
    rounded as (S + 128) >> 8 (round half up).
  * Gauss rows 0, 1, H-2, H-1 are copied unfiltered; in the other rows a
    neighbour column outside the frame takes the nearest in-frame column.
  * Thres: output 255 where |a - b| > T (strict), else 0, with a the
    current and b the previous Gauss output; the initial token is an
    all-zero frame.
  * Med: median of the plus-shaped set {centre, up, down, left, right}; a
    neighbour outside the frame takes the nearest in-frame pixel.
Exact integer arithmetic throughout.
"""
from __future__ import annotations

import numpy as np

from .dataflow import Actor, Fifo, Scheduler, Sink, Source

# 5-tap binomial row (Pascal's triangle, row 4); the 2-D kernel is its outer product.
BINOMIAL5 = np.array([1, 4, 6, 4, 1], np.int64)
GAUSS_KERNEL = np.outer(BINOMIAL5, BINOMIAL5)          # sums to 256


def _clamped(frame: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """frame[y+dy, x+dx] with out-of-frame coordinates moved to the nearest
    in-frame row/column."""
    H, W = frame.shape
    ys = np.clip(np.arange(H) + dy, 0, H - 1)
    xs = np.clip(np.arange(W) + dx, 0, W - 1)
    return frame[ys][:, xs]


def gauss5(frame: np.ndarray) -> np.ndarray:
    """Gauss firing on one frame (Sec. 4.1): 5x5 binomial filter, rounded
    (S + 128) >> 8, rows 0, 1, H-2, H-1 copied unfiltered."""
    f = np.asarray(frame, np.uint8)
    H, W = f.shape
    s = np.zeros((H, W), np.int64)
    for i, dy in enumerate(range(-2, 3)):
        for j, dx in enumerate(range(-2, 3)):
            s += GAUSS_KERNEL[i, j] * _clamped(f, dy, dx).astype(np.int64)
    out = ((s + 128) >> 8).astype(np.uint8)
    keep = np.zeros(H, bool)
    keep[:2] = True
    keep[max(H - 2, 0):] = True
    out[keep] = f[keep]
    return out


def thres(cur: np.ndarray, prev: np.ndarray, threshold: int) -> np.ndarray:
    """Thres firing (Sec. 4.1): 255 where |cur - prev| > threshold, else 0."""
    d = np.abs(np.asarray(cur, np.int64) - np.asarray(prev, np.int64))
    return np.where(d > threshold, 255, 0).astype(np.uint8)


def med5(frame: np.ndarray) -> np.ndarray:
    """Med firing (Sec. 4.1): median of the plus-shaped 5-pixel neighbourhood,
    out-of-frame neighbours replaced by the nearest in-frame pixel."""
    f = np.asarray(frame, np.uint8)
    stack = np.stack([_clamped(f, dy, dx) for dy, dx in ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1))])
    return np.sort(stack, axis=0)[2].astype(np.uint8)


class Gauss(Actor):
    def fire(self, consumed, token):
        g = np.stack([gauss5(f) for f in consumed["in"]]) if len(consumed["in"]) else consumed["in"]
        return {"cur": g, "delayed": g.copy()}


class Thres(Actor):
    def __init__(self, name, threshold):
        super().__init__(name)
        self.threshold = threshold

    def fire(self, consumed, token):
        out = [thres(c, p, self.threshold) for c, p in zip(consumed["cur"], consumed["prev"])]
        return {"out": np.stack(out)}


class Med(Actor):
    def fire(self, consumed, token):
        return {"out": np.stack([med5(f) for f in consumed["in"]])}


class PaperMotionNetwork:
    """Src -> Gauss -> {cur, delayed (1 initial token)} -> Thres -> Med -> Sink,
    every channel at token rate ``rate`` (Sec. 4.1; 4 on the GPU)."""

    def __init__(self, frames, threshold=20, rate=4):
        frames = np.asarray(frames, np.uint8)
        n, H, W = frames.shape
        shp = (H, W)
        self.f_in = Fifo("in", shp, np.uint8, rate)
        self.f_cur = Fifo("g_cur", shp, np.uint8, rate)
        self.f_del = Fifo("g_delayed", shp, np.uint8, rate, n_initial=1)
        self.f_thr = Fifo("thr", shp, np.uint8, rate)
        self.f_out = Fifo("out", shp, np.uint8, rate)
        self.src = Source("Src", {"in": frames})
        self.src.connect_out("in", self.f_in)
        self.gauss = Gauss("Gauss")
        self.gauss.connect_in("in", self.f_in)
        self.gauss.connect_out("cur", self.f_cur)
        self.gauss.connect_out("delayed", self.f_del)
        self.thres = Thres("Thres", threshold)
        self.thres.connect_in("cur", self.f_cur)
        self.thres.connect_in("prev", self.f_del)
        self.thres.connect_out("out", self.f_thr)
        self.med = Med("Med")
        self.med.connect_in("in", self.f_thr)
        self.med.connect_out("out", self.f_out)
        self.sink = Sink("Sink")
        self.sink.connect_in("out", self.f_out)
        self.sched = Scheduler([self.src, self.gauss, self.thres, self.med, self.sink])

    def run(self, policy="round_robin", seed=0):
        self.sched.run(policy=policy, seed=seed)
        return self.sink.collected("out")


def run_paper_motion(frames, threshold=20, rate=4, policy="round_robin", seed=0):
    """Output frames of the network: one per input frame, up to the last
    whole firing (a multiple of ``rate``)."""
    return PaperMotionNetwork(frames, threshold, rate).run(policy, seed)


def paper_motion_direct(frames, threshold=20, prev_gauss=None):
    """Closed form of the network's output stream: frame k maps to
    med5(thres(gauss5(f_k), gauss5(f_{k-1}))), with gauss5(f_{-1}) taken
    from ``prev_gauss`` (the initial token, all-zero by default)."""
    frames = np.asarray(frames, np.uint8)
    prev = np.zeros(frames.shape[1:], np.uint8) if prev_gauss is None else np.asarray(prev_gauss, np.uint8)
    out = np.zeros_like(frames)
    for k, f in enumerate(frames):
        g = gauss5(f)
        out[k] = med5(thres(g, prev, threshold))
        prev = g
    return out
