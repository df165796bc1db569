"""FP64 CPU oracle (test infrastructure only; never imported by the product path).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  It shares no code with the GPU path.
"""
from .core import *  # noqa: F401,F403
