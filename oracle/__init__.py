"""FP64 CPU oracle for the PRISM analysis-by-synthesis pass.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.
"""
from .prism_oracle import *  # noqa: F401,F403
from .prism_oracle import Constants, Problem, TERMS  # noqa: F401
