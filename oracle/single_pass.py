"""The single-pass eigenvalue decomposition of a Hermitian matrix (Section 5.5), in FP64 on the CPU.

TEST INFRASTRUCTURE (see the package docstring): only tests, the smoke check
and the benchmark's CPU-baseline leg use this module.

Algorithm 5.6 (eigenvalue decomposition in one pass): A is touched once, by the
sample Y = A Omega.  Since B = Q* A Q satisfies B (Q* Omega) ~ Q* Y when
A ~ A Q Q* (the relation of Section 5.5), B is found from Omega, Y and Q alone
by least squares, then B = V Lambda V*, U = Q V.  The remark that closes
Section 5.5 improves the conditioning of that system by oversampling: with
Omega of k + p columns, Q is the n x k matrix of the k leading left singular
vectors of Y, and the system B (Q* Omega) ~ Q* Y for the k x k matrix B is
overdetermined (k x (k + p) coefficient matrix).

Readings where the paper is silent:
  * "A standard least-squares solver to find an Hermitian matrix": the
    standard (unconstrained) least-squares solution of B M = N with
    M = Q* Omega, N = Q* Y, i.e. B M M* = N M* (M has full row rank), then its
    Hermitian part (B + B*)/2.
  * p = 0 (no oversampling): Q = an orthonormal basis of range(Y) (the square
    system of the algorithm box); p > 0: the remark's k leading left singular
    vectors.
  * The k eigenpairs are returned in decreasing order of |lambda| (equal
    magnitudes: the positive one first), like Algorithm 5.3.

Library primitives stand in for single steps only: numpy products, Householder
QR and SVD (LAPACK), numpy's least-squares solver and Hermitian eigensolver.
"""

import numpy as np

from .herm import hermitian_part
from .rsvd import adj, qr_pos


def one_pass_basis(Y, k):
    """Q for Algorithm 5.6: the k leading left singular vectors of Y (k < columns of Y), or an
    orthonormal basis of range(Y) (k == columns of Y)."""
    if k == Y.shape[1]:
        Q, _ = qr_pos(Y)
        return Q
    U, _, _ = np.linalg.svd(Y, full_matrices=False)
    return U[:, :k]


def least_squares_core(Q, Omega, Y):
    """Step 1: B with B (Q* Omega) ~ Q* Y in the least-squares sense, made Hermitian."""
    M = adj(Q) @ Omega
    N = adj(Q) @ Y
    # B M = N  <=>  M* B* = N*: a standard least-squares problem for the columns of B*
    Bs, *_ = np.linalg.lstsq(adj(M), adj(N), rcond=None)
    return hermitian_part(adj(Bs))


def one_pass_eig(A, Omega, k):
    """Algorithm 5.6 with the oversampling of the closing remark: returns (U (n x k), lam (k,))."""
    Y = A @ Omega  # the one pass over A
    Q = one_pass_basis(Y, k)
    B = least_squares_core(Q, Omega, Y)
    lam, V = np.linalg.eigh(B)
    order = sorted(range(lam.size), key=lambda i: (-abs(lam[i]), -lam[i]))
    return Q @ V[:, order], lam[order]
