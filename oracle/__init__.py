"""FP64 CPU oracle of the free-mesh transform -- test infrastructure only.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The GPU library never calls it.
"""
from .fmt_oracle import *  # noqa: F401,F403
from .fmt_oracle import __all__  # noqa: F401
