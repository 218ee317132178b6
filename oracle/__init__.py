"""FP64 CPU oracle for the randomized SVD hot path (Halko, Martinsson, Tropp).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plainly written reference
that the GPU path is checked against.  Only the test suite, the smoke check of
the package entry point and the CPU-baseline leg of the benchmark may import
it.  The product library (the C ABI and its Python binding) never imports,
links or calls anything in here, and shares no code with it.

Contents
--------
philox      Counter-based generator (Philox4x64-10, published by Salmon, Moraes,
            Dror and Shaw, SC'11) and the draws the method makes from it: the
            Gaussian test matrix of Algorithm 4.1 and the SRFT ingredients of
            the SRFT definition in Section 4.6.
rsvd        The method itself, step by step in FP64 with LAPACK (through numpy)
            for Householder QR and dense SVD: Algorithms 4.1, 4.3, 4.4, 4.5 and
            5.1, the truncation of Remark 5.1, and the prototype randomized SVD
            of Section 1.6.
adaptive    The fixed-precision range finder: Algorithm 4.2 one sample at a time
            and in blocks of doubling size, with the a posteriori estimate of
            eq. (4.3) as its stopping test (Sections 4.3-4.4).
herm        Stage B for Hermitian and positive semidefinite A: Algorithm 5.3
            (direct eigenvalue decomposition) and Algorithm 5.5 (Nystrom).
single_pass The eigenvalue decomposition of a Hermitian matrix in one pass over it:
            Algorithm 5.6 with the oversampled basis of the closing remark of
            Section 5.5; the two-sided single pass for a general matrix.
gsrft       The test matrix built from chains of random Givens rotations (the
            remark on random Givens rotations in Section 4.6), real form.
row_extraction  Stage B by row extraction: the interpolative decomposition of the
            basis and Algorithm 5.2.
evaluate    Residual norms ||A - QQ*A|| and ||A - U S V*|| and the paper's error
            bounds (Theorems 9.1-9.3, 10.5, 10.6, Corollaries 10.9, 10.10).
rsvd_grad   The reference gradient of the fixed-Omega randomized SVD: the same
            forward map in plain PyTorch CPU FP64, differentiated by autograd
            (the paper defines no derivative; this is the FP64 reference the
            hand-written adjoint is compared with).

Every function is pinned by a CPU test (tests/test_oracle_*.py) against
something other than itself: numpy's own Philox, brute-force DFTs and SVDs,
exact-rank recovery and the deterministic theorems of Section 9.
"""

from . import philox, rsvd, evaluate, adaptive, herm, single_pass, gsrft, row_extraction  # noqa: F401
# rsvd_grad imports torch; it is imported on its own where needed.
