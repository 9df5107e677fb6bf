"""FP64 CPU oracle of the PnP-ULA sampler -- test infrastructure only.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product library neither imports it
nor shares any code with it.
"""
from .oracle import *  # noqa: F401,F403
