"""Seeded synthetic inputs for the randomized SVD: matrices with prescribed spectra.

This module builds test inputs only.  It holds none of the method's
arithmetic (no sketch, no orthonormalization of samples, no projection), so
both the GPU path and the CPU oracle can be fed from it.  The random test
matrix Omega that the method itself draws is NOT made here: each side draws it
from its own implementation of the counter-based generator.

Construction: A = U diag(sigma) V^T with U (m x r) and V (n x r), r = min(m, n),
the Q factors (with positive diag R) of seeded standard Gaussian matrices, so
U and V are Haar-distributed and the singular values of A are exactly sigma in
exact arithmetic.  The paper's own experiments (Section 7) use operators and
datasets that are not available here; these matrices stand in for them, with
spectra that decay fast (exponential), slowly (1/j, j^-1/2) or have a gap.
"""

from .matrices import (  # noqa: F401
    CONFIGS, Config, spectrum, haar_factor, build_matrix, build_matrix_torch,
    batch_shapes, grad_targets, SEED, build_symmetric, build_psd_torch,
)
