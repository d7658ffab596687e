"""CPU oracle for parallel intersection-free QEM simplification (TEST INFRASTRUCTURE).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product path (the HIP library and its binding) never
imports, links or calls anything under ``oracle/``.
"""
from .oracle import *  # noqa: F401,F403
