"""Plain CPU oracle for the SCALP clustering path (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product path never does.
"""
from .oracle import *  # noqa: F401,F403
