"""CPU FP64 oracle for the RLB-MIE-FD Allen-Cahn scheme (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library.
"""
from .oracle import *  # noqa: F401,F403
