"""FP64 CPU oracle for the SNAP hot path (TEST INFRASTRUCTURE).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The HIP library never imports, links or calls it, and it
imports nothing of the HIP library.
"""
from .snap_oracle import *  # noqa: F401,F403
from . import snap_oracle  # noqa: F401
