"""Channel sizing of Sec. 3.2.  TEST INFRASTRUCTURE ONLY.

Eq. (1): a channel of token rate r and token size S bytes holds S*(3r+1)
bytes when it carries a delay token (the buffer of Fig. 2: the delay token in
slot 0, writes of r tokens to slots 1..3r in turn, and after the write that
reaches slot 3r a copy of slot 3r to slot 0, so every read of r tokens is
contiguous), and S*2r bytes otherwise (a double buffer).
"""
from __future__ import annotations


def capacity_tokens(rate: int, has_delay: bool) -> int:
    """Token capacity of a channel by Eq. (1)."""
    if rate < 1:
        raise ValueError("token rate must be a positive integer")
    return 3 * rate + 1 if has_delay else 2 * rate


def capacity_bytes(token_bytes: int, rate: int, has_delay: bool) -> int:
    """Bytes of a channel by Eq. (1): S_f times its token capacity."""
    return int(token_bytes) * capacity_tokens(rate, has_delay)


def network_bytes(channels) -> int:
    """Total channel memory of a network given (token_bytes, rate, has_delay)
    per channel, as tabulated in Table 1."""
    return sum(capacity_bytes(s, r, d) for s, r, d in channels)


def paper_motion_channels(width: int = 320, height: int = 240, rate: int = 4):
    """The channels of the motion-detection network of Sec. 4.1 (Src -> Gauss,
    Gauss -> Thres twice, one with the delay token, Thres -> Med,
    Med -> Sink), one frame per token."""
    s = width * height
    return [(s, rate, False), (s, rate, False), (s, rate, True), (s, rate, False), (s, rate, False)]
