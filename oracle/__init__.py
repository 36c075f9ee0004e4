"""FP64 CPU oracle of the Domain Transform Solver (Bapat & Frahm, ECCV 2018).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's
CPU-baseline leg, never by the product path.  It shares no code with the HIP library.
"""
from .dts_oracle import *  # noqa: F401,F403
from .dts_oracle import __all__  # noqa: F401
