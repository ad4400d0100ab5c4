"""Oracle for the motion-detection network.  TEST INFRASTRUCTURE ONLY.

Sec. 4.1 builds motion detection from consecutive-frame subtraction with a
fixed threshold, where the previous frame reaches the subtracting actor over
a channel holding one initial token (a one-frame delay).  This network keeps
that idiom and uses the actor body this library implements:

    Src -> cur  (no initial token)  -> Detect -> mask  -> Gate -> mask_out  -> Sink
        -> prev (1 initial token)   ->        -> count -> (Gate's control port)
                                                         -> index_out -> Sink

Detect (static, rate 1 everywhere): D = |cur - prev| in integers; a pixel is
changed iff D > threshold; the mask is opened: 3x3 erosion, then 3x3
dilation, where neighbours outside the frame are ignored (erosion treats them
as set, dilation as clear).  It emits the mask as 255/0 bytes and the number
of set pixels of the opened mask as Gate's control token.

Gate (dynamic): its control token is the count; its mask input always has
rate 1; both outputs (the mask and the int64 frame index) have rate 1 iff
1000 * count >= permille * W * H, else 0 - a frame with too few changed
pixels produces no output tokens.

The initial token on ``prev`` is an all-zero frame.  Exact integer arithmetic.
"""
from __future__ import annotations

import numpy as np

from .dataflow import Actor, Fifo, Scheduler, Sink, Source


def threshold_mask(cur: np.ndarray, prev: np.ndarray, threshold: int) -> np.ndarray:
    """Changed iff |cur - prev| > threshold (strict), computed in int16."""
    d = np.abs(cur.astype(np.int16) - prev.astype(np.int16))
    return d > threshold


def erode3x3(m: np.ndarray) -> np.ndarray:
    """AND over the in-frame 3x3 neighbourhood (out-of-frame counts as set)."""
    H, W = m.shape
    p = np.ones((H + 2, W + 2), bool)
    p[1:-1, 1:-1] = m
    out = np.ones((H, W), bool)
    for dy in range(3):
        for dx in range(3):
            out &= p[dy:dy + H, dx:dx + W]
    return out


def dilate3x3(m: np.ndarray) -> np.ndarray:
    """OR over the in-frame 3x3 neighbourhood (out-of-frame counts as clear)."""
    H, W = m.shape
    p = np.zeros((H + 2, W + 2), bool)
    p[1:-1, 1:-1] = m
    out = np.zeros((H, W), bool)
    for dy in range(3):
        for dx in range(3):
            out |= p[dy:dy + H, dx:dx + W]
    return out


def detect(cur, prev, threshold=25):
    """Detect's firing: (opened mask as 0/255 uint8, changed-pixel count)."""
    o = dilate3x3(erode3x3(threshold_mask(cur, prev, threshold)))
    return o.astype(np.uint8) * np.uint8(255), int(o.sum())


def emits(count: int, width: int, height: int, permille: int = 1) -> bool:
    """Gate's rate rule: outputs have rate 1 iff 1000*count >= permille*W*H."""
    return 1000 * int(count) >= int(permille) * width * height


class Detect(Actor):
    def __init__(self, name, threshold):
        super().__init__(name)
        self.threshold = threshold

    def fire(self, consumed, token):
        mask, count = detect(consumed["cur"][0], consumed["prev"][0], self.threshold)
        return {"mask": mask[None], "count": np.array([count], np.int64)}


class Gate(Actor):
    def __init__(self, name, width, height, permille):
        super().__init__(name)
        self.W, self.H, self.permille = width, height, permille
        self.frame = 0

    def control(self, token):
        k = 1 if emits(token, self.W, self.H, self.permille) else 0
        return {"mask": 1}, {"mask_out": k, "index_out": k}

    def fire(self, consumed, token):
        t = self.frame
        self.frame += 1
        if emits(token, self.W, self.H, self.permille):
            return {"mask_out": consumed["mask"], "index_out": np.array([t], np.int64)}
        return {}


class MotionNetwork:
    def __init__(self, frames, threshold=25, permille=1):
        frames = np.asarray(frames, np.uint8)
        n, H, W = frames.shape
        self.fcur = Fifo("cur", (H, W), np.uint8, 1)
        self.fprev = Fifo("prev", (H, W), np.uint8, 1, n_initial=1)
        self.fmask = Fifo("mask", (H, W), np.uint8, 1)
        self.fcount = Fifo("count", (), np.int64, 1)
        self.fout = Fifo("mask_out", (H, W), np.uint8, 1)
        self.fidx = Fifo("index_out", (), np.int64, 1)
        self.src = Source("Src", {"cur": frames, "prev": frames})
        self.src.connect_out("cur", self.fcur)
        self.src.connect_out("prev", self.fprev)
        self.det = Detect("Detect", threshold)
        self.det.connect_in("cur", self.fcur)
        self.det.connect_in("prev", self.fprev)
        self.det.connect_out("mask", self.fmask)
        self.det.connect_out("count", self.fcount)
        self.gate = Gate("Gate", W, H, permille)
        self.gate.connect_ctrl(self.fcount)
        self.gate.connect_in("mask", self.fmask)
        self.gate.connect_out("mask_out", self.fout)
        self.gate.connect_out("index_out", self.fidx)
        self.sink = Sink("Sink")
        self.sink.connect_in("mask_out", self.fout)
        self.sink.connect_in("index_out", self.fidx)
        self.sched = Scheduler([self.src, self.det, self.gate, self.sink])

    def run(self, policy="round_robin", seed=0):
        self.sched.run(policy=policy, seed=seed)
        return self.sink.collected("mask_out"), self.sink.collected("index_out")


def run_motion(frames, threshold=25, permille=1, policy="round_robin", seed=0):
    """(masks uint8 [k][H][W], frame indices int64 [k]) for the emitted frames."""
    return MotionNetwork(frames, threshold, permille).run(policy, seed)


def frame_counts(frames, threshold=25) -> np.ndarray:
    """Opened-mask count of every frame against its predecessor (frame 0
    against the all-zero initial token)."""
    frames = np.asarray(frames, np.uint8)
    prev = np.zeros_like(frames[0])
    out = np.zeros(len(frames), np.int64)
    for t, f in enumerate(frames):
        out[t] = detect(f, prev, threshold)[1]
        prev = f
    return out
