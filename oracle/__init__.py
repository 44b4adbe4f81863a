"""FP64 CPU oracle of the DDGI-resampling hot path.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the HIP implementation (see gi_oracle.c for the method
readings it follows).
"""
from .ref import *  # noqa: F401,F403
