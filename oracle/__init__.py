"""Plain, slow, obviously-correct FP64 CPU oracle for the MSP hot path.

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import it. The product path (the C-ABI library and
its Python binding) never calls into it and shares no code with it.

Modules
    rng      SplitMix64 (Steele, Lea, Flood 2014) and the sparse-embedding index draw
    sketch   the sparse embedding matrix of Definition 2.1 and its products
    krylov   flexible PCG (used at every level) and Algorithm 6 (preconditioned Lanczos)
    msp      Algorithms 1-2 (two-level, PSD) and 3-5 (three-level, general)
    refine   FP64 iterative refinement around a low-precision MSP solve
    trace    Schatten-p / effective-dimension estimation through ridge solves (Section 3.2)
    dense    plain definitions of every final result (dense solves, spectral sums, gradients)

Parity status: every function has a pin in ``tests/test_oracle_*.py`` (closed forms,
library routines, brute force on tiny inputs or the paper's worked examples).
"""
from . import rng, sketch, krylov, msp, refine, trace, dense  # noqa: F401
