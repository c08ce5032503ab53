"""Plain FP64 CPU oracle of the pseudo-spectral penalized Navier-Stokes hot path.

TEST INFRASTRUCTURE ONLY. This package is a slow, obviously-correct reference
written from the paper (Engels, Kolomenskiy, Schneider, Sesterhenn, "FluSI",
arXiv:1506.06513).  Only the test-suite, the smoke check of the entry module
and the CPU-baseline leg of the benchmark may import it.  It shares no code
with the HIP library and must never be used as a fallback by the product path.
"""
from .flusi_oracle import *  # noqa: F401,F403
