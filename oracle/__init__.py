"""CPU oracle for the HWSDA hot path -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package. The product path (paper_2511_01255_amd) never does.
"""
from .oracle import *  # noqa: F401,F403
