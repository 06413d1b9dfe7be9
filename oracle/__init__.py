"""FP64 CPU oracle of the LLOID filtering core.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library (paper_2511_04730_amd) and does not import it.
"""
from .lloid import *  # noqa: F401,F403
