"""CPU FP64 oracle for the EGFEM Newton hot path (test infrastructure only).

Used by the tests, the smoke check and the CPU-baseline leg of the benchmark;
never by the product path."""
from .egfem_oracle import *  # noqa: F401,F403
