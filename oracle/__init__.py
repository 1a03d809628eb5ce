"""FP64 CPU oracle for DEANN's query path (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library.
"""
from .deann_ref import *  # noqa: F401,F403
from .deann_ref import GAUSSIAN, EXPONENTIAL  # noqa: F401
