"""CPU float64 oracle for the CTD hot path.

TEST INFRASTRUCTURE ONLY: tests/, the package smoke check and the benchmark's
CPU-baseline leg may import it; the product path never does.  Shares no code
with the HIP library.
"""
from . import ctd, philox  # noqa: F401
