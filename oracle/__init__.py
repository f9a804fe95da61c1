"""CPU FP64 oracle for the direct domain-decomposition solver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or call anything in this package; the
solver itself never does, and shares no code with it.
"""
from .dd_oracle import (arrowhead, cond1_estimate, dense_solve, dual_blocks, global_residual, global_solve,
                        interface_inverse, rel_error, serial_dd, torn_residual)

__all__ = ["arrowhead", "cond1_estimate", "dense_solve", "dual_blocks", "global_residual", "global_solve",
           "interface_inverse", "rel_error", "serial_dd", "torn_residual"]
