"""FP64 CPU oracle for randomized HOSVD / R-STHOSVD.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package.  Only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark use
it.  It shares no code with the GPU implementation: the two are written
independently against the same published definitions (the paper's
algorithms, and the Philox4x32-10 generator of Salmon et al., SC'11).

Everything here is deliberately plain: NumPy arrays in float64, LAPACK QR
and SVD through numpy.linalg, one library call per algorithmic step, in the
order the paper states the steps.  Speed is not a goal.

Modules
-------
philox      Philox4x32-10, the 24-bit uniform map and Box-Muller; the Gaussian
            test matrices Omega used by every sketch.
tensor_ops  n-unfolding, folding and the mode-n product (Section 2).
rsvd        Basic randomized SVD with oversampling and power iteration
            (Algorithm 1, Section 3.1).
tucker      Deterministic THOSVD / STHOSVD (Section 4, Algorithm 4) and the
            randomized RP-HOSVD (Algorithm 6) and R-STHOSVD (Algorithm 8),
            plus the relative error of Section 8.
variants    Fixed-precision (adaptive-rank) R-STHOSVD (Section 5.1), RP-HOOI
            (Algorithm 7) and R-PET (Algorithm 9).

Parity status: every function is pinned by the CPU tests in
tests/test_oracle_*.py (published known-answer vectors, an independent
library implementation, closed forms, invariants and brute-force SVD on
tiny inputs); none is "parity unpinned".
"""
from . import philox, tensor_ops, rsvd, tucker, variants  # noqa: F401
