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
  * The Hermitian B of step 1, asked of an ordinary least-squares solver: the
    unconstrained least-squares solution of B M = N with
    M = Q* Omega, N = Q* Y, i.e. B M M* = N M* (M has full row rank), then its
    Hermitian part (B + B*)/2.
  * p = 0 (no oversampling): Q = an orthonormal basis of range(Y) (the square
    system of the algorithm box); p > 0: the remark's k leading left singular
    vectors.
  * The k eigenpairs are returned in decreasing order of |lambda| (equal
    magnitudes: the positive one first), like Algorithm 5.3.

The same section sketches a single pass for a general A: Y = A Omega and
Yt = A* Omegat in one pass, orthonormal bases Q and Qt of their ranges, and the
reduced matrix B = Q* A Qt determined as the minimum-residual solution of its
two relations B (Qt* Omega) ~ Q* Y and B* (Q* Omegat) ~ Qt* Yt
(two_sided_svd; its SVD then gives U = Q Ub, V = Qt Vb).

Library primitives stand in for single steps only: numpy products, Householder
QR and SVD (LAPACK), numpy's least-squares solver and Hermitian eigensolver,
scipy's Sylvester solver (the normal-equation route to the two-sided core).
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


# ---------------------------------------------------------------------------
# The two-sided single pass for a general A (Section 5.5, after Algorithm 5.6)
# ---------------------------------------------------------------------------

def two_sided_core(M1, N1, M2, N2):
    """The minimum-residual B of the two relations of Section 5.5:
        B M1 ~ N1   (M1 = Qt* Omega,  N1 = Q* Y)
        B* M2 ~ N2  (M2 = Q* Omegat, N2 = Qt* Yt)
    i.e. argmin_B ||B M1 - N1||_F^2 + ||B* M2 - N2||_F^2, as one linear least-squares problem in the
    entries of B (numpy's lstsq on the stacked, vectorized relations)."""
    l, lt = N1.shape[0], M1.shape[0]  # B is l x lt
    # row-major vec: vec(B M1) = kron(I_l, M1^T) vec(B); vec(B^T M2) = kron(M2^T, I_lt) P vec(B) with
    # P the l x lt -> lt x l transposition, written out entry by entry
    rows1 = np.kron(np.eye(l), M1.T)
    T = np.zeros((l * lt, l * lt))
    for i in range(l):
        for j in range(lt):
            T[j * l + i, i * lt + j] = 1.0
    rows2 = np.kron(np.eye(lt), M2.T) @ T
    Asys = np.vstack([rows1, rows2])
    rhs = np.concatenate([N1.reshape(-1), N2.reshape(-1)])
    b, *_ = np.linalg.lstsq(Asys, rhs, rcond=None)
    return b.reshape(l, lt)


def two_sided_core_normal(M1, N1, M2, N2):
    """The same minimizer from its normal equations (the gradient of the objective set to zero):
        B (M1 M1*) + (M2 M2*) B = N1 M1* + M2 N2*,
    a Sylvester equation, solved by scipy's Bartels-Stewart solver.  For large l, where the stacked
    system of two_sided_core (2 l^2 x l^2) is too slow; squares the conditioning of the relations."""
    from scipy.linalg import solve_sylvester
    return solve_sylvester(M2 @ adj(M2), M1 @ adj(M1), N1 @ adj(M1) + M2 @ adj(N2))


def two_sided_svd(A, Omega, Omegat, k, solver="lstsq"):
    """The single-pass factorization of a general A: Y = A Omega and Yt = A* Omegat (one pass over A),
    Y = Q R and Yt = Qt Rt (orthonormal bases), B from the two least-squares relations, B = Ub S Vb*,
    U = Q Ub, V = Qt Vb, truncated to k.  Returns (U (m x k), S (k,), V (n x k)).  solver: "lstsq"
    (two_sided_core) or "normal" (two_sided_core_normal, for large l)."""
    Y = A @ Omega
    Yt = adj(A) @ Omegat
    Q, R = qr_pos(Y)
    Qt, Rt = qr_pos(Yt)
    core = two_sided_core if solver == "lstsq" else two_sided_core_normal
    B = core(adj(Qt) @ Omega, adj(Q) @ Y, adj(Q) @ Omegat, adj(Qt) @ Yt)
    Ub, S, Vbh = np.linalg.svd(B, full_matrices=False)
    return (Q @ Ub)[:, :k], S[:k], (Qt @ adj(Vbh))[:, :k]
