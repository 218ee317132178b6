"""The structured test matrix built from chains of random Givens rotations (the
remark on random Givens rotations in Section 4.6), in FP64 on the CPU.

TEST INFRASTRUCTURE (see the package docstring): only tests, the smoke check
and the benchmark's CPU-baseline leg use this module.

The remark proposes Omega = D'' Theta' D' Theta D F R, where D, F, R are the
SRFT's (random signs, Fourier matrix, column sampler), D' and D'' are further
independent random diagonals, and each Theta = Pi G(1, 2; theta_1) ...
G(n-1, n; theta_{n-1}) is a random permutation followed by a chain of rotations
in consecutive coordinate planes with independent angles uniform on [0, 2 pi).

Readings where the paper is silent:
  * Real tailoring, as for the SRFT sketch of this library: D' and D'' are
    random +-1 diagonals, the rotations are real, and D F R is the real SRFT
    (sqrt(n/l) D F_r R with F_r the real orthonormal Fourier basis), so
    Omega = D'' Theta' D' Theta (sqrt(n/l) D F_r R).
  * G(i, k; theta) is the rotation of Golub and Van Loan's Section 5.1.8:
    the identity except G_ii = G_kk = c, G_ik = s, G_ki = -s (c = cos theta,
    s = sin theta); a row vector x times G(i, k) has entries
    (x G)_i = c x_i - s x_k and (x G)_k = s x_i + c x_k.
  * The permutation matrix acts on row vectors as a gather: (x Pi)_j = x_pi(j)
    (Pi_ij = 1 exactly when i = pi(j)).
  * The draws follow the generator contract of oracle.philox (chain 0: D',
    Theta; chain 1: D'', Theta').

Library primitives: numpy products and indexing, and the SRFT sketch of
oracle.rsvd for the final D F_r R.
"""

import numpy as np

from . import philox
from .rsvd import qr_pos, real_srft_sketch, real_srft_test_matrix


def rotation_chain_rows(X, theta):
    """Rows of X times G(1, 2; theta_1) G(2, 3; theta_2) ... G(n-1, n; theta_{n-1}), applied one
    rotation after the other (0-based: the rotation j acts in the plane (j, j + 1))."""
    Y = np.array(X, dtype=np.float64, copy=True)
    for j, th in enumerate(theta):
        c, s = np.cos(th), np.sin(th)
        a, b = Y[:, j].copy(), Y[:, j + 1].copy()
        Y[:, j] = c * a - s * b
        Y[:, j + 1] = s * a + c * b
    return Y


def givens_factor_rows(X, d, pi, theta):
    """Rows of X times D Theta = D Pi G(1, 2) ... G(n-1, n), D = diag(d)."""
    XD = np.asarray(X, dtype=np.float64) * d[None, :]
    return rotation_chain_rows(XD[:, pi], theta)


def draws(n, seed, stream=0):
    """The GSRFT's random parts beyond the SRFT's: ((d', pi, theta), (d'', pi', theta'))."""
    return tuple((philox.givens_signs(n, seed, c, stream), philox.givens_permutation(n, seed, c, stream),
                  philox.givens_angles(n, seed, c, stream)) for c in (0, 1))


def pretransform_rows(A, seed, stream=0):
    """A D'' Theta' D' Theta: the part of the GSRFT in front of the SRFT's D F_r R."""
    (d0, p0, t0), (d1, p1, t1) = draws(A.shape[1], seed, stream)
    return givens_factor_rows(givens_factor_rows(A, d1, p1, t1), d0, p0, t0)


def gsrft_sketch(A, l, seed, stream=0):
    """Y = A Omega for the real GSRFT Omega = D'' Theta' D' Theta (sqrt(n/l) D F_r R) (m x l)."""
    n = A.shape[1]
    d = philox.srft_signs(n, seed, stream)
    R = philox.srft_sample(n, l, seed, stream)
    return real_srft_sketch(pretransform_rows(A, seed, stream), d, R)


def gsrft_test_matrix(n, l, seed, stream=0):
    """The dense n x l Omega, from the pretransform of the identity; O(n^2), small n only."""
    T = pretransform_rows(np.eye(n), seed, stream)
    d = philox.srft_signs(n, seed, stream)
    R = philox.srft_sample(n, l, seed, stream)
    return T @ real_srft_test_matrix(n, d, R)


def gsrft_range_finder(A, l, seed, stream=0):
    """Algorithm 4.1 with the GSRFT test matrix: Q, an orthonormal basis of range(A Omega)."""
    Q, _ = qr_pos(gsrft_sketch(A, l, seed, stream))
    return Q
