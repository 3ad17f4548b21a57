"""Plain FP64 CPU oracle of the Keldysh bubble / SDE / susceptibility / multiloop path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark; never by the product path.  It shares no code
with the HIP library.
"""
from .oracle import *  # noqa: F401,F403
