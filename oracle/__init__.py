"""CPU FP64 oracle for reverse k-MIPS top-N (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The library never does, and this package imports
nothing from the library.
"""
from .reference import *  # noqa: F401,F403
from .reference import __all__  # noqa: F401
