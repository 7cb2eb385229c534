"""CPU oracle for colour-coding tree counting -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding) must
never import, link or execute anything here.
"""
from .oracle import *  # noqa: F401,F403
