"""Dataflow core of the oracle: FIFO channels, actors, sequential scheduler.

Follows Sec. 2.2 (network of actors and FIFO channels, token rates, static
and dynamic actors, the dynamic firing rule, initial tokens) and Sec. 3.1
(``control`` runs once per firing right before ``fire`` and fixes every
regular port's rate to 0 or r for that firing).  TEST INFRASTRUCTURE ONLY.

A token is one row of a numpy array; a channel holds tokens of one shape and
dtype.  Reads and writes move whole tokens in FIFO order.  The scheduler fires
exactly one actor at a time.
"""
from __future__ import annotations

from collections import deque
import random

import numpy as np


class Fifo:
    """Order-preserving channel connecting one output port to one input port
    (Sec. 3.2).  ``rate`` is the channel's token rate r (Sec. 2.2); ports
    adopt it.  ``initial`` are the initial (delay) tokens present before any
    firing (Sec. 2.2); the paper allows 0 or 1, here any number (the
    generalisation Sec. 3.2 mentions and omits).  ``capacity`` None means
    unbounded."""

    def __init__(self, name: str, token_shape=(), dtype=np.complex128, rate: int = 1,
                 initial=None, n_initial: int = 0, capacity: int | None = None):
        if rate < 1:
            raise ValueError("token rate must be a positive integer")
        self.name = name
        self.token_shape = tuple(token_shape)
        self.dtype = np.dtype(dtype)
        self.rate = int(rate)
        self.capacity = capacity
        self._chunks: deque[np.ndarray] = deque()
        self._count = 0
        self.n_written = 0          # tokens written by the producer (initial excluded)
        self.n_read = 0             # tokens consumed by the reader
        self.writer = None
        self.reader = None
        if initial is None and n_initial:
            initial = np.zeros((n_initial,) + self.token_shape, self.dtype)
        self.n_initial = 0 if initial is None else int(len(initial))
        if self.n_initial:
            self._push(np.asarray(initial, self.dtype))

    # -- raw storage
    def _push(self, arr: np.ndarray) -> None:
        if len(arr):
            self._chunks.append(np.array(arr, dtype=self.dtype, copy=True))
            self._count += len(arr)

    def count(self) -> int:
        return self._count

    def space(self) -> float:
        return float("inf") if self.capacity is None else self.capacity - self._count

    def write(self, tokens) -> None:
        tokens = np.asarray(tokens, dtype=self.dtype)
        if tokens.shape[1:] != self.token_shape:
            raise ValueError(f"{self.name}: token shape {tokens.shape[1:]} != {self.token_shape}")
        if self.capacity is not None and self._count + len(tokens) > self.capacity:
            raise RuntimeError(f"{self.name}: write of {len(tokens)} tokens overflows")
        self._push(tokens)
        self.n_written += len(tokens)

    def peek(self, k: int) -> np.ndarray:
        if k > self._count:
            raise RuntimeError(f"{self.name}: peek {k} of {self._count}")
        out, need = [], k
        for c in self._chunks:
            if need == 0:
                break
            take = min(need, len(c))
            out.append(c[:take])
            need -= take
        if not out:
            return np.zeros((0,) + self.token_shape, self.dtype)
        return np.concatenate(out)

    def read(self, k: int) -> np.ndarray:
        if k > self._count:
            raise RuntimeError(f"{self.name}: read {k} of {self._count}")
        out, need = [], k
        while need:
            c = self._chunks[0]
            if len(c) <= need:
                out.append(self._chunks.popleft())
                need -= len(c)
            else:
                out.append(c[:need])
                self._chunks[0] = c[need:]
                need = 0
        self._count -= k
        self.n_read += k
        if not out:
            return np.zeros((0,) + self.token_shape, self.dtype)
        return np.concatenate(out)


class Actor:
    """Actor with regular input/output ports and, if dynamic, one control
    input port of rate 1 (Sec. 2.2).  Subclasses implement ``control`` (Sec.
    3.1: maps one control token to the rate, 0 or r, of every regular port
    for this firing) and ``fire`` (consumed tokens -> produced tokens).
    Static actors have no control port and fixed rates.  ``init``/``finish``
    of Sec. 3.1 are the constructor and nothing, respectively."""

    dynamic = False

    def __init__(self, name: str):
        self.name = name
        self.inputs: dict[str, Fifo] = {}
        self.outputs: dict[str, Fifo] = {}
        self.ctrl: Fifo | None = None
        self.n_fired = 0

    # wiring -----------------------------------------------------------
    def connect_in(self, port: str, f: Fifo) -> None:
        if f.reader is not None:
            raise RuntimeError(f"{f.name} already has a reader")
        f.reader = (self, port)
        self.inputs[port] = f

    def connect_out(self, port: str, f: Fifo) -> None:
        if f.writer is not None:
            raise RuntimeError(f"{f.name} already has a writer")
        f.writer = (self, port)
        self.outputs[port] = f

    def connect_ctrl(self, f: Fifo) -> None:
        if f.rate != 1:
            raise ValueError("a control port has token rate 1")
        if f.n_initial:
            raise ValueError("initial tokens are not allowed on a control channel")
        if f.reader is not None:
            raise RuntimeError(f"{f.name} already has a reader")
        f.reader = (self, "ctrl")
        self.ctrl = f
        self.dynamic = True

    # behaviour --------------------------------------------------------
    def control(self, token):
        """Return ({in_port: rate}, {out_port: rate}) for this firing."""
        return ({p: f.rate for p, f in self.inputs.items()},
                {p: f.rate for p, f in self.outputs.items()})

    def fire(self, consumed: dict, token) -> dict:
        raise NotImplementedError

    def exhausted(self) -> bool:
        """Sources override this: True when nothing is left to emit."""
        return True


class Source(Actor):
    """Source actor: no input ports; each firing emits the next ``rate``
    tokens of a fixed token sequence on every output port ``port``."""

    def __init__(self, name: str, port_data: dict):
        super().__init__(name)
        self.port_data = {p: np.asarray(v) for p, v in port_data.items()}
        self.pos = {p: 0 for p in port_data}

    def control(self, token):
        out = {}
        for p, f in self.outputs.items():
            left = len(self.port_data[p]) - self.pos[p]
            out[p] = f.rate if left >= f.rate else 0
        return {}, out

    def fire(self, consumed, token):
        res = {}
        for p, f in self.outputs.items():
            k = f.rate if len(self.port_data[p]) - self.pos[p] >= f.rate else 0
            res[p] = self.port_data[p][self.pos[p]:self.pos[p] + k]
            self.pos[p] += k
        return res

    def exhausted(self) -> bool:
        return all(len(self.port_data[p]) - self.pos[p] < self.outputs[p].rate
                   for p in self.port_data)


class Sink(Actor):
    """Sink actor: no output ports; consumes ``rate`` tokens per firing from
    every input and keeps them in order."""

    def __init__(self, name: str):
        super().__init__(name)
        self.received: dict[str, list] = {}

    def fire(self, consumed, token):
        for p, v in consumed.items():
            self.received.setdefault(p, []).append(v)
        return {}

    def collected(self, port: str, fifo: Fifo | None = None) -> np.ndarray:
        chunks = self.received.get(port, [])
        if chunks:
            return np.concatenate(chunks)
        f = fifo or self.inputs[port]
        return np.zeros((0,) + f.token_shape, f.dtype)


class Scheduler:
    """Sequential scheduler: repeatedly picks one fireable actor and fires it,
    until no actor is fireable (quiescence).

    fireable(a): a dynamic actor needs one control token, which is peeked and
    mapped by ``control`` to this firing's port rates; every regular input
    must then hold at least its rate and every bounded output must have room
    (blocking reads and writes, Sec. 2.2).  A Source fires while it has data.
    fire(a): consume the control token, consume each input at its fixed rate,
    run ``fire``, produce each output at its fixed rate (Sec. 2.2)."""

    def __init__(self, actors):
        self.actors = list(actors)
        self.trace: list[str] = []

    def _rates(self, a: Actor):
        if a.dynamic:
            if a.ctrl.count() < 1:
                return None
            tok = a.ctrl.peek(1)[0]
            return (tok,) + tuple(a.control(tok))
        rin, rout = a.control(None)
        return (None, rin, rout)

    def fireable(self, a: Actor) -> bool:
        r = self._rates(a)
        if r is None:
            return False
        _, rin, rout = r
        if isinstance(a, Source):
            if not any(rout.values()):
                return False
        elif not a.inputs and not a.dynamic:
            return False                      # would fire forever
        for p, k in rin.items():
            if a.inputs[p].count() < k:
                return False
        for p, k in rout.items():
            if a.outputs[p].space() < k:
                return False
        return True

    def fire(self, a: Actor) -> None:
        tok, rin, rout = self._rates(a)
        if a.dynamic:
            a.ctrl.read(1)
        consumed = {p: a.inputs[p].read(k) for p, k in rin.items()}
        produced = a.fire(consumed, tok)
        for p, k in rout.items():
            v = produced.get(p)
            n = 0 if v is None else len(v)
            if n != k:
                raise RuntimeError(f"{a.name}.{p}: produced {n} tokens, rate is {k}")
            if k:
                a.outputs[p].write(v)
        a.n_fired += 1
        self.trace.append(a.name)

    def run(self, policy: str = "round_robin", seed: int = 0,
            max_firings: int | None = None) -> int:
        """Fire until quiescent.  policy "round_robin" scans actors in id order
        and fires every fireable one per sweep; "random" picks one fireable
        actor uniformly (seeded).  Returns the number of firings."""
        rng = random.Random(seed)
        n = 0
        while max_firings is None or n < max_firings:
            if policy == "round_robin":
                progressed = False
                for a in self.actors:
                    if self.fireable(a):
                        self.fire(a)
                        n += 1
                        progressed = True
                        if max_firings is not None and n >= max_firings:
                            return n
                if not progressed:
                    break
            elif policy == "random":
                cands = [a for a in self.actors if self.fireable(a)]
                if not cands:
                    break
                self.fire(rng.choice(cands))
                n += 1
            else:
                raise ValueError(policy)
        return n

    def blocked(self) -> list[str]:
        """Deadlock report at quiescence.

        A channel is closed when its writer has finished: an exhausted
        source, or (by fixpoint) an actor that cannot fire because some
        closed input no longer holds a firing's worth of tokens.  An actor
        is blocked when it cannot fire, some input (or its control channel)
        that starves it is still open, and it holds tokens it cannot use.
        Leftover tokens at the end of a finite stream (short of one firing,
        or circulating in a feedback loop) are therefore not a deadlock.
        A non-empty list after ``run`` means the network deadlocked."""
        closed = set()
        for a in self.actors:
            if isinstance(a, Source) and a.exhausted():
                closed.update(id(f) for f in a.outputs.values())
        finished = set()
        changed = True
        while changed:
            changed = False
            for a in self.actors:
                if isinstance(a, Source) or id(a) in finished or self.fireable(a):
                    continue
                chans = list(a.inputs.values()) + ([a.ctrl] if a.ctrl is not None else [])
                if any(id(f) in closed and f.count() < f.rate for f in chans):
                    finished.add(id(a))
                    closed.update(id(f) for f in a.outputs.values())
                    changed = True
        out = []
        for a in self.actors:
            if isinstance(a, Source):
                if not a.exhausted():
                    out.append(a.name)
                continue
            if id(a) in finished or self.fireable(a):
                continue
            pending = (a.ctrl is not None and a.ctrl.count() > 0) or \
                any(f.count() >= f.rate for f in a.inputs.values())
            if pending:
                out.append(a.name)
        return out
