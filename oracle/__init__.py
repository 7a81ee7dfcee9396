"""Serial FP64 CPU oracle for the LDU pressure solve (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library.
"""
from .oracle import *  # noqa: F401,F403
