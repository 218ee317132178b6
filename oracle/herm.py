"""Stage B for Hermitian and positive semidefinite matrices (Sections 5.3-5.4), in FP64 on the CPU.

TEST INFRASTRUCTURE (see the package docstring): only tests, the smoke check
and the benchmark's CPU-baseline leg use this module.

Given a Hermitian A (n x n) and a basis Q (n x l) with orthonormal columns, such
as the range finders of Section 4 return:

  * direct_eig follows Algorithm 5.3 (direct eigenvalue decomposition):
    B = Q* A Q, B = V Lambda V*, U = Q V.  Section 5.3 bounds its error (all
    l terms kept): ||A - U Lambda U*|| <= 2 ||A - Q Q* A||.
  * nystrom_eig follows Algorithm 5.5 (eigenvalue decomposition by the Nystrom
    method) for positive semidefinite A: B1 = A Q, B2 = Q* B1 = C* C (Cholesky,
    C upper triangular), F = B1 C^-1 (a triangular solve), F = U Sigma V*,
    Lambda = Sigma^2.  Then U Lambda U* = F F* = (AQ)(Q*AQ)^-1(AQ)*, the
    Nystrom approximation of Section 5.4, whose error never exceeds
    ||A - Q Q* A|| (the lemma of Drineas and Mahoney that Section 5.4 cites).

Readings where the paper is silent:
  * B = Q*AQ and B2 = Q*B1 are Hermitian in exact arithmetic only; both are
    replaced by their Hermitian part (B + B*)/2 before the eigendecomposition or
    the Cholesky factorization.
  * Truncation to rank k (Section 5 keeps the leading terms): Algorithm 5.3
    keeps the k eigenpairs of largest |lambda|, ordered by decreasing |lambda|
    (equal magnitudes: the positive one first); Algorithm 5.5 keeps the k
    largest lambda = sigma^2, in decreasing order.
  * Algorithm 5.5 needs B2 positive definite.  When B2 is singular to working
    precision the paper gives no rule: this oracle factors whatever B2 rounding
    leaves (numpy raises LinAlgError only on a pivot that is not positive), and
    the cases it is compared on keep B2 well conditioned.

Library primitives stand in for single steps only: numpy products, numpy's
Hermitian eigensolver and Cholesky (LAPACK), scipy's triangular solve and
numpy's SVD.
"""

import numpy as np
import scipy.linalg

from .rsvd import adj


def hermitian_part(B):
    """(B + B*) / 2."""
    return 0.5 * (B + adj(B))


def direct_eig(A, Q, k):
    """Algorithm 5.3 truncated to k terms: returns (U (n x k), lam (k,)).

    Step 1: B = Q* A Q.  Step 2: B = V Lambda V* (Hermitian eigensolver).
    Step 3: U = Q V.  The k eigenpairs of largest |lambda| are kept, ordered by
    decreasing |lambda|.
    """
    B = hermitian_part(adj(Q) @ (A @ Q))
    lam, V = np.linalg.eigh(B)
    order = sorted(range(lam.size), key=lambda i: (-abs(lam[i]), -lam[i]))[:k]
    U = Q @ V[:, order]
    return U, lam[order]


def nystrom_factor(A, Q):
    """Steps 1-3 of Algorithm 5.5: the approximate Cholesky factor F (n x l) of Section 5.4."""
    B1 = A @ Q
    B2 = hermitian_part(adj(Q) @ B1)
    L = np.linalg.cholesky(B2)  # B2 = L L*, so C = L* is the upper factor of B2 = C* C
    C = adj(L)
    # F = B1 C^-1  <=>  C* F* = B1*  (lower triangular system with L = C*)
    F = adj(scipy.linalg.solve_triangular(L, adj(B1), lower=True))
    return F, C


def nystrom_eig(A, Q, k):
    """Algorithm 5.5 truncated to k terms: returns (U (n x k), lam (k,)).

    Step 4: F = U Sigma V*, Lambda = Sigma^2; the k largest kept.
    """
    F, _ = nystrom_factor(A, Q)
    U, s, _ = np.linalg.svd(F, full_matrices=False)
    return U[:, :k], s[:k] ** 2
