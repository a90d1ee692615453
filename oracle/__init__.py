"""FP64 CPU oracle of the binary-lens fitness and the evolutionary algorithm.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the library's
product path never does.  It shares no code with the HIP implementation.
"""
from .oracle import *  # noqa: F401,F403
