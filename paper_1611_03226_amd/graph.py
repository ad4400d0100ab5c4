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

    def set_tile(self, tile=0, k=0, bpc=0):
        D.df_set_tile(self.g, tile, k, bpc)

    # builders -------------------------------------------------------------
    def dpd_chain(self, h, r, n_delay=0, initial=None, history="branch", cap_x=0, cap_ctrl=0,
                  cap_y=0) -> DPDChain:
        h = np.ascontiguousarray(h, np.complex64)
        B, M = h.shape
        p = D.DpdParams(B, M, r, h.ctypes.data, 0,
                        D.DF_HIST_SHARED if history == "shared" else D.DF_HIST_BRANCH)
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
