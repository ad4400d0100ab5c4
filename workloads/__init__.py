"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the bench.

This package only draws inputs (signals, control tokens, coefficients,
frames).  It holds none of the method's arithmetic: no basis functions, no
filtering of actor outputs, no morphology.  Both the CPU oracle and the HIP
path consume exactly these arrays.
"""
from .gen import *  # noqa: F401,F403
