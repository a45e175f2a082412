"""CPU oracle of the frame-to-event simulator (TEST INFRASTRUCTURE ONLY).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this package.  The
product library never loads it and shares no code with it.
"""
from .oracle import (OracleSim, accumulate, build, event_rate, lut, run_sequence,  # noqa: F401
                     lk_flow, BASIC, DENSE, SPARSE, DIFFERENCE, LOG, LINEAR, REFERENCE,
                     MEMORYLESS, FLOW_SUPPLIED, FLOW_LK)
