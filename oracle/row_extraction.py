"""Stage B by row extraction (Algorithm 5.2, Section 5.2), in FP64 on the CPU.

TEST INFRASTRUCTURE (see the package docstring): only tests, the smoke check
and the benchmark's CPU-baseline leg use this module.  No GPU code computes this
yet; the oracle comes first.

The interpolative decomposition (Section 3.2.3) of the basis: Q = X Q(J,:) with
J a set of k row indices and X an m x k matrix with X(J,:) = I_k.  Since
A ~ Q Q* A = X Q(J,:) Q* A and Q(J,:) Q* A ~ A(J,:), A ~ X A(J,:): k rows of A
and no product with A.  Algorithm 5.2 turns that into an SVD: A(J,:) = R* W*
(a QR factorization of A(J,:)*), Z = X R*, Z = U Sigma Vt*, V = W Vt.

Readings where the paper is silent or garbled:
  * The ID is computed by a column-pivoted (Businger-Golub) QR of Q* (k x m):
    J = the first k pivots, X(J,:) = I, and the other rows of X from
    R11^-1 R12.  The paper asks for entries of X bounded by two, which a
    strong rank-revealing QR guarantees; plain column pivoting keeps them small
    in practice, and the tests check the bound on their inputs rather than
    assume it.
  * The lemma's final bound reads [1 + sqrt(1 + 4k(n - k))] eps, but X is
    m x k and its rows outside J number m - k: read as
    [1 + sqrt(1 + 4k(m - k))] eps.  The bound its proof establishes first,
    (1 + ||X||) eps, holds for any ID with X(J,:) = I and is the one pinned.
  * The remark after the algorithm prefers the sample matrix Y to Q for the
    ID (Y = X Y(J,:)); both are offered (`basis`).

Library primitives: scipy's column-pivoted QR, numpy's QR, SVD and triangular
solve (through solve).
"""

import numpy as np
from scipy.linalg import qr as scipy_qr, solve_triangular

from .rsvd import adj


def row_id(B):
    """Row ID of an m x k matrix B of rank k: B = X B(J,:), X(J,:) = I.  Returns (J, X)."""
    m, k = B.shape
    _, R, piv = scipy_qr(adj(B), mode="economic", pivoting=True)
    J = piv[:k]
    # B* P = Qr [R11 R12]  =>  B* = B*(:, J) [I, R11^-1 R12] P*  =>  B = P [I; (R11^-1 R12)*] B(J,:)
    T = solve_triangular(R[:k, :k], R[:k, k:])
    X = np.zeros((m, k), dtype=np.result_type(B, np.float64))
    X[J, :] = np.eye(k)
    X[piv[k:], :] = adj(T)
    return J, X


def extract_rows_svd(A, B):
    """Algorithm 5.2 with the ID taken of B (the basis Q, or the sample matrix Y): returns
    (U (m x k), S (k,), V (n x k), J, X)."""
    J, X = row_id(B)
    AJ = A[J, :]                                 # step 2: k rows of A
    W, R = np.linalg.qr(adj(AJ))                 # A(J,:)* = W R, i.e. A(J,:) = R* W*
    Z = X @ adj(R)                               # step 3
    U, S, Vth = np.linalg.svd(Z, full_matrices=False)  # step 4
    V = W @ adj(Vth)                             # step 5
    return U, S, V, J, X
