"""Convenience wrapper over the C ABI for building small networks.

Graph owns one df_graph; dpd_chain / motion_chain create an actor together
with the channels it reads and writes (the host is the source and the sink).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import dfhip as D


def _pow2(n: int) -> int:
    p = 1
    while p < n:
        p <<= 1
    return p


@dataclass
class DPDChain:
    actor: int
    ctrl: int      # int32 control channel (host writes)
    x: int         # complex64 input channel (host writes)
    y: int         # complex64 output channel (host reads)
    r: int
    n_branches_max: int
    n_taps: int


@dataclass
class MotionChain:
    actor: int
    cur: int
    prev: int      # -1 with self_delay
    mask: int
    index: int
    width: int
    height: int


@dataclass
class PaperMotionPipeline:
    """Src -> Gauss -> {cur, delayed} -> Thres -> Med -> Sink (Sec. 4.1)."""
    gauss: int
    thres: int
    med: int
    inp: int       # host writes frames
    g_cur: int     # Gauss -> Thres
    g_delayed: int # Gauss -> Thres, one initial (all-zero) token
    thr: int       # Thres -> Med
    out: int       # host reads frames
    width: int
    height: int
    rate: int

    def fire_all(self, G: "Graph", n_firings: int) -> None:
        """Fire each actor n_firings times, in pipeline order (three launches)."""
        for a in (self.gauss, self.thres, self.med):
            G.fire(a, n_firings)

    def fire_chain(self, G: "Graph", n_firings: int, fused: bool = True, partial: bool = False) -> int:
        """The same firings through df_fire_pipeline (one fused launch when it applies)."""
        flags = (0 if fused else D.DF_PIPE_SEPARATE) | (D.DF_FIRE_PARTIAL if partial else 0)
        return D.df_fire_pipeline(G.g, self.gauss, self.thres, self.med, n_firings, flags)


class Graph:
    def __init__(self, device: int = 0, stream=None):
        self.g = D.df_graph_create(device, stream)

    def close(self) -> None:
        if self.g:
            D.df_graph_destroy(self.g)
            self.g = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # thin forwards --------------------------------------------------------
    def fifo(self, dtype, elems_per_token=1, capacity=0, n_initial=0, initial=None) -> int:
        return D.df_fifo_create(self.g, dtype, elems_per_token, capacity, n_initial, initial)

    def push(self, fifo, data, n=None):
        D.df_push(self.g, fifo, data, n)

    def pop(self, fifo, dst, n=None) -> int:
        return D.df_pop(self.g, fifo, dst, n)

    def fire(self, actor, n, partial=False) -> int:
        return D.df_fire(self.g, actor, n, D.DF_FIRE_PARTIAL if partial else 0)

    def fire_many(self, actors, n_firings, persistent=False, graph=False):
        flags = (D.DF_FIRE_PERSISTENT if persistent else 0) | (D.DF_FIRE_GRAPH if graph else 0)
        D.df_fire_many(self.g, actors, n_firings, flags)

    def status(self, fifo):
        return D.df_fifo_status(self.g, fifo)

    def sync(self):
        D.df_sync(self.g)

    def profile(self, enable=True):
        D.df_profile_enable(self.g, enable)

    def profile_read(self, actor=None):
        if actor is None:
            return D.df_profile_read(self.g)
        return D.df_profile_read_actor(self.g, actor)

    def set_tile(self, tile=0, k=0, bpc=0):
        D.df_set_tile(self.g, tile, k, bpc)

    # builders -------------------------------------------------------------
    def dpd_chain(self, h, r, n_delay=0, initial=None, history="branch", cap_x=0, cap_ctrl=0,
                  cap_y=0, control="count") -> DPDChain:
        """A predistortion actor with its control, input and output channels;
        control="mask" reads control tokens as bit masks of active branches."""
        h = np.ascontiguousarray(h, np.complex64)
        B, M = h.shape
        if control not in ("count", "mask"):
            raise ValueError(f"unknown control mode {control!r}")
        p = D.DpdParams(B, M, r, h.ctypes.data, 0,
                        D.DF_HIST_SHARED if history == "shared" else D.DF_HIST_BRANCH,
                        D.DF_CTRL_MASK if control == "mask" else D.DF_CTRL_COUNT, 0)
        a = D.df_actor_create(self.g, D.DF_ACTOR_DPD, p)
        fc = self.fifo(D.DF_I32, 1, cap_ctrl)
        fx = self.fifo(D.DF_C64, 1, cap_x, n_delay, initial)
        fy = self.fifo(D.DF_C64, 1, cap_y)
        D.df_connect(self.g, a, D.DF_DPD_CTRL, fc)
        D.df_connect(self.g, a, D.DF_DPD_IN, fx)
        D.df_connect(self.g, a, D.DF_DPD_OUT, fy)
        return DPDChain(a, fc, fx, fy, r, B, M)

    def motion_chain(self, width, height, threshold=25, permille=1, self_delay=True, cap_in=0,
                     cap_out=0) -> MotionChain:
        p = D.MotionParams(width, height, threshold, permille, 1 if self_delay else 0)
        a = D.df_actor_create(self.g, D.DF_ACTOR_MOTION, p)
        wh = width * height
        fc = self.fifo(D.DF_U8, wh, cap_in or 16)
        fp = -1
        if not self_delay:
            fp = self.fifo(D.DF_U8, wh, cap_in or 16, 1)       # one zero initial frame
            D.df_connect(self.g, a, D.DF_MD_PREV, fp)
        fm = self.fifo(D.DF_U8, wh, cap_out or 16)
        fi = self.fifo(D.DF_I64, 1, cap_out or 16)
        D.df_connect(self.g, a, D.DF_MD_CUR, fc)
        D.df_connect(self.g, a, D.DF_MD_MASK, fm)
        D.df_connect(self.g, a, D.DF_MD_INDEX, fi)
        return MotionChain(a, fc, fp, fm, fi, width, height)

    def paper_motion_pipeline(self, width, height, threshold=20, rate=4, cap=0,
                              second_output=True, cap_io=0, layout="ring") -> PaperMotionPipeline:
        """Gauss, Thres and Med actors with their five channels; the three
        inner channels hold ``cap`` frames (0: 16), the host-facing input and
        output channels ``cap_io`` (0: same as cap).  With
        second_output=False Gauss writes one channel only and Thres's
        previous-frame channel must be fed by the caller.  layout="paper"
        builds every channel in the paper's layout instead (Eq. (1): double
        buffers of 2*rate frames, the delay channel 3*rate + 1 frames with
        the Fig. 2 access pattern); batches then hold at most two firings."""
        wh = width * height
        p = D.FrameParams(width, height, rate, threshold)
        ga = D.df_actor_create(self.g, D.DF_ACTOR_GAUSS5, p)
        ta = D.df_actor_create(self.g, D.DF_ACTOR_THRES, p)
        ma = D.df_actor_create(self.g, D.DF_ACTOR_MED5, p)
        if layout == "paper":
            def pf(n_initial=0):
                return D.df_fifo_create_paper(self.g, D.DF_U8, wh, rate, n_initial)
            f_in, f_cur, f_del, f_thr, f_out = pf(), pf(), pf(1), pf(), pf()
        elif layout == "ring":
            c = cap or 16
            cio = cap_io or c
            f_in = self.fifo(D.DF_U8, wh, cio)
            f_cur = self.fifo(D.DF_U8, wh, c)
            f_del = self.fifo(D.DF_U8, wh, c, 1)         # the one-frame delay
            f_thr = self.fifo(D.DF_U8, wh, c)
            f_out = self.fifo(D.DF_U8, wh, cio)
        else:
            raise ValueError(f"unknown layout {layout!r}")
        D.df_connect(self.g, ga, D.DF_GAUSS_IN, f_in)
        D.df_connect(self.g, ga, D.DF_GAUSS_OUT, f_cur)
        if second_output:
            D.df_connect(self.g, ga, D.DF_GAUSS_OUT2, f_del)
        D.df_connect(self.g, ta, D.DF_THRES_CUR, f_cur)
        D.df_connect(self.g, ta, D.DF_THRES_PREV, f_del)
        D.df_connect(self.g, ta, D.DF_THRES_OUT, f_thr)
        D.df_connect(self.g, ma, D.DF_MED_IN, f_thr)
        D.df_connect(self.g, ma, D.DF_MED_OUT, f_out)
        return PaperMotionPipeline(ga, ta, ma, f_in, f_cur, f_del, f_thr, f_out, width, height, rate)
