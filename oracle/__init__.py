"""FP64 CPU oracle for the warm-started SR step.

Test infrastructure: imported only by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code with
the HIP library and imports nothing from it.
"""
from .wssr_oracle import *  # noqa: F401,F403
