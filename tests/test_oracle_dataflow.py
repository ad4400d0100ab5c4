"""Pins for the oracle's FIFO channels and scheduler (CPU only).

FIFO order and initial tokens are pinned to the paper's worked delay-token
buffer (Sec. 3.2, Fig. 2: tests/golden/fig2_delay_token_r4.txt), the
scheduler to Kahn determinacy across random schedules and to a feedback
network that is an IIR filter (Sec. 2.2: initial tokens model feedback).
"""
import os

import numpy as np
import pytest
import scipy.signal

from oracle.dataflow import Actor, Fifo, Scheduler, Sink, Source

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _parse_fig2():
    ops = []
    slots = None
    initial = None
    with open(os.path.join(GOLDEN, "fig2_delay_token_r4.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            if line[0] == "slots":
                slots = int(line[1])
            elif line[0] == "initial":
                initial = int(line[1])
            else:
                op = (line[0], int(line[1]), int(line[2]),
                      (int(line[4]), int(line[5])) if len(line) > 3 else None)
                ops.append(op)
    return slots, initial, ops


def test_fig2_delay_buffer_order_matches_fifo_with_one_initial_token():
    """Run the paper's delay-token buffer for several cycles on labelled
    tokens; its read sequence must be the FIFO order with one initial token."""
    slots, initial, ops = _parse_fig2()
    r = 4
    assert slots == 3 * r + 1          # Eq. (1), delay-token case
    buf = [None] * slots
    buf[initial] = "D"
    written = iter(range(10 ** 6))
    reads = []
    for _cycle in range(5):
        for op, lo, hi, copy in ops:
            assert hi - lo + 1 == r
            if op == "write":
                for s in range(lo, hi + 1):
                    buf[s] = next(written)
                if copy:
                    buf[copy[1]] = buf[copy[0]]
            else:
                reads.extend(buf[lo:hi + 1])
    f = Fifo("f", (), object, rate=r, initial=np.array(["D"], object))
    n_written = sum(1 for op in ops if op[0] == "write") * 5 * r
    f.write(np.array(list(range(n_written)), object))
    fifo_reads = list(f.read(len(reads)))
    assert fifo_reads == reads
    assert reads[:4] == ["D", 0, 1, 2]       # first read = D + first r-1 tokens


@pytest.mark.parametrize("d", [0, 1, 3])
def test_fifo_order_initial_tokens_and_conservation(d):
    rng = np.random.default_rng(0)
    init = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    f = Fifo("f", (), np.complex128, rate=3, initial=init)
    data = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    out = []
    pos = 0
    for k in [5, 1, 7, 0, 20, 17]:
        f.write(data[pos:pos + k])
        pos += k
        take = int(rng.integers(0, f.count() + 1))
        out.append(f.read(take))
        # written + initial - read == occupancy
        assert f.n_written + d - f.n_read == f.count()
    out.append(f.read(f.count()))
    got = np.concatenate(out)
    assert np.array_equal(got, np.concatenate([init, data]))


def test_fifo_bounds_and_wiring_errors():
    f = Fifo("f", (), np.int64, rate=2, capacity=4)
    f.write([1, 2, 3, 4])
    with pytest.raises(RuntimeError):
        f.write([5])
    with pytest.raises(RuntimeError):
        f.read(5)
    a, b = Actor("a"), Actor("b")
    a.connect_in("i", f)
    with pytest.raises(RuntimeError):
        b.connect_in("i", f)                 # exactly one reader (Sec. 3.2)
    c = Fifo("c", (), np.int64, rate=1, n_initial=1)
    with pytest.raises(ValueError):
        b.connect_ctrl(c)                    # no initial tokens on a control channel
    with pytest.raises(ValueError):
        b.connect_ctrl(Fifo("c2", (), np.int64, rate=2))   # control rate is 1


class _Add(Actor):
    """Static two-input adder with feedback scaling: y = x + a*fb."""

    def __init__(self, name, a):
        super().__init__(name)
        self.a = a

    def fire(self, consumed, token):
        y = consumed["x"] + self.a * consumed["fb"]
        return {"y": y, "loop": y}


def _iir_network(x, a, with_delay):
    fx = Fifo("x", (), np.float64, 1)
    fb = Fifo("fb", (), np.float64, 1, n_initial=1 if with_delay else 0)
    fy = Fifo("y", (), np.float64, 1)
    src = Source("src", {"x": x})
    src.connect_out("x", fx)
    add = _Add("add", a)
    add.connect_in("x", fx)
    add.connect_in("fb", fb)
    add.connect_out("y", fy)
    add.connect_out("loop", fb)
    sink = Sink("sink")
    sink.connect_in("y", fy)
    return Scheduler([src, add, sink]), sink


def test_feedback_with_initial_token_is_an_iir_filter():
    """Sec. 2.2: initial tokens model feedback such as IIR filters.
    y[n] = x[n] + 0.5 y[n-1] must equal scipy.signal.lfilter."""
    x = np.random.default_rng(1).standard_normal(40)
    sched, sink = _iir_network(x, 0.5, True)
    sched.run()
    assert sched.blocked() == []
    want = scipy.signal.lfilter([1.0], [1.0, -0.5], x)
    np.testing.assert_allclose(sink.collected("y"), want, rtol=0, atol=1e-12)


def test_feedback_without_initial_token_deadlocks():
    x = np.arange(5.0)
    sched, sink = _iir_network(x, 0.5, False)
    n = sched.run()
    assert n == 5                              # only the source fired
    assert "add" in sched.blocked()
    assert len(sink.collected("y")) == 0


def test_random_schedules_give_identical_streams():
    x = np.random.default_rng(2).standard_normal(64)
    ref = None
    for policy, seed in [("round_robin", 0), ("random", 1), ("random", 2), ("random", 3)]:
        sched, sink = _iir_network(x, -0.25, True)
        sched.run(policy=policy, seed=seed)
        y = sink.collected("y")
        if ref is None:
            ref = y
        assert np.array_equal(ref, y)
