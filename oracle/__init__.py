"""FP64 CPU oracle for AMGF-preconditioned CG (test infrastructure only).

This package is the slow, plain reference that the GPU library is checked against.
Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product path never does.  It shares no code with the HIP library:
its only dependency inside the repository is the seeded input generator.
"""
from .amgf_oracle import (  # noqa: F401
    BlockMatrix, OracleOptions, OracleAMGF, schur_operator, strength_graph,
    fmix32, mis2_sequential, aggregate, gram_schmidt_qr, pcg,
)
