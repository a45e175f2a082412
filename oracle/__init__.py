"""CPU oracle of the frame-to-event simulator (TEST INFRASTRUCTURE ONLY).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this package.  The
product library never loads it and shares no code with it.
"""
from .oracle import OracleSim, build, lut, run_sequence, BASIC, DENSE, SPARSE, LOG, LINEAR  # noqa: F401
