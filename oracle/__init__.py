"""FP64 CPU oracle for the Hermite-regularized LBM step (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never does.
"""
from .oracle import *  # noqa: F401,F403
