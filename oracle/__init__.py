"""FP64 CPU reference for the EPIC imaging path (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it and shares no code with
it; the two meet only through the seeded inputs in ``synth``.
"""
from .epic_oracle import *  # noqa: F401,F403
from .fixed_point import *  # noqa: F401,F403
