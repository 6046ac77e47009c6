"""FP64 CPU oracle for the gMCO / gL-BFGS method.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute anything in this package: only the test-suite, the smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code with the HIP
library and reads its inputs from the seeded generators in ``cases``.
"""
from .gmco_oracle import *  # noqa: F401,F403
