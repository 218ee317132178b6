"""Pins of the Hermitian / psd Stage B oracle (oracle/herm.py), Sections 5.3-5.4.

1. Algorithm 5.3, exact case: for a symmetric A of rank r <= l (eigenvalues of both signs) and a
   basis Q with range(A) inside range(Q), U Lambda U^T = A and the kept eigenvalues are the r
   prescribed ones in the stated order (largest magnitude first, a negative one leading when its
   magnitude is largest); U is orthonormal.
2. Algorithm 5.3, the bound of Section 5.3: with all l terms kept,
   ||(I - QQ*)A|| <= ||A - U Lambda U*|| <= 2 ||(I - QQ*)A||
   (the left side holds because (I - QQ*) kills Q B Q*), on decaying spectra with Q from the range
   finder of Algorithm 4.1.
3. Algorithm 5.5, exact case: for a psd A and Q = V_l W (the top-l eigenvectors times an arbitrary
   orthogonal W), the Nystrom factor gives exactly the top-l eigenpairs: lambda = the top
   eigenvalues, U Lambda U^T = the best rank-k approximation of A.
4. Algorithm 5.5, the bounds of Section 5.4: ||A - F F*|| <= ||(I - QQ*)A|| (the error never
   exceeds the basis error), and A - F F* is positive semidefinite (F F* = A^1/2 P A^1/2 with P the
   orthogonal projector onto range(A^1/2 Q)); with k = l, U Lambda U* = F F*, and the factor C is
   upper triangular with C^T C = Q^T A Q.
A dropped term, a wrong transpose or a wrong ordering in either algorithm fails one of these.
"""

import numpy as np
import pytest

from oracle import herm, rsvd
from workloads import build_symmetric


def _range_basis(A, l, seed):
    Om = rsvd.gaussian_test_matrix(A.shape[1], l, seed)
    return rsvd.randomized_range_finder(A, Om)


def _orth_err(U):
    return np.linalg.norm(U.T @ U - np.eye(U.shape[1]), 2)


@pytest.mark.parametrize("n,lam,l", [
    (60, [5.0, -7.0, 3.0, -1.0, 0.5], 8),
    (90, [-2.0, 2.0, 1.0, -0.25, 4.0, 0.125, -3.5], 7),
])
def test_direct_eig_exact_range(n, lam, l):
    A = build_symmetric(n, lam, seed=11)
    Q = _range_basis(A, l, seed=12)
    U, got = herm.direct_eig(A, Q, len(lam))
    expect = sorted(lam, key=lambda x: (-abs(x), -x))
    assert np.allclose(got, expect, rtol=0, atol=1e-12 * max(abs(x) for x in lam))
    assert np.linalg.norm(A - (U * got[None, :]) @ U.T, 2) <= 1e-12 * np.linalg.norm(A, 2)
    assert _orth_err(U) <= 1e-13
    # U spans the eigenvectors: A U = U Lambda
    assert np.linalg.norm(A @ U - U * got[None, :], 2) <= 1e-12 * np.linalg.norm(A, 2)


@pytest.mark.parametrize("kind,seed", [("exp", 21), ("inv", 22), ("signed", 23)])
def test_direct_eig_two_epsilon_bound(kind, seed):
    n, l = 120, 12
    j = np.arange(1, n + 1, dtype=np.float64)
    lam = {"exp": np.exp(-j / 4.0), "inv": 1.0 / j, "signed": (-1.0) ** j / j}[kind]
    A = build_symmetric(n, lam, seed=seed)
    Q = _range_basis(A, l, seed=seed + 100)
    eps = np.linalg.norm(A - Q @ (Q.T @ A), 2)
    U, got = herm.direct_eig(A, Q, l)
    err = np.linalg.norm(A - (U * got[None, :]) @ U.T, 2)
    assert eps * (1 - 1e-12) <= err <= 2 * eps * (1 + 1e-12)
    assert _orth_err(U) <= 1e-13
    # the order: nonincreasing magnitude
    assert np.all(np.diff(np.abs(got)) <= 1e-15)


@pytest.mark.parametrize("n,l,k", [(80, 10, 6), (64, 16, 16)])
def test_nystrom_exact_top_eigenspace(n, l, k):
    j = np.arange(1, n + 1, dtype=np.float64)
    lam = 1.0 / j ** 1.5
    A, V = build_symmetric(n, lam, seed=31, return_factors=True)
    W, _ = np.linalg.qr(np.random.default_rng(32).standard_normal((l, l)))
    Q = V[:, :l] @ W
    U, got = herm.nystrom_eig(A, Q, k)
    assert np.allclose(got, lam[:k], rtol=1e-12, atol=0)
    Ak = (V[:, :k] * lam[None, :k]) @ V[:, :k].T
    assert np.linalg.norm((U * got[None, :]) @ U.T - Ak, 2) <= 1e-12 * lam[0]
    assert _orth_err(U) <= 1e-13


@pytest.mark.parametrize("decay,seed", [(0.5, 41), (1.0, 42), (2.0, 43)])
def test_nystrom_bounds(decay, seed):
    n, l = 150, 14
    j = np.arange(1, n + 1, dtype=np.float64)
    lam = j ** -decay
    A = build_symmetric(n, lam, seed=seed)
    Q = _range_basis(A, l, seed=seed + 100)
    eps = np.linalg.norm(A - Q @ (Q.T @ A), 2)
    F, C = herm.nystrom_factor(A, Q)
    nA = np.linalg.norm(A, 2)
    E = A - F @ F.T
    assert np.linalg.norm(E, 2) <= eps * (1 + 1e-10)
    assert np.min(np.linalg.eigvalsh(0.5 * (E + E.T))) >= -1e-12 * nA
    assert np.allclose(np.tril(C, -1), 0.0)
    assert np.linalg.norm(C.T @ C - Q.T @ A @ Q, 2) <= 1e-12 * nA
    U, got = herm.nystrom_eig(A, Q, l)
    assert np.linalg.norm((U * got[None, :]) @ U.T - F @ F.T, 2) <= 1e-12 * nA
    assert np.all(got >= 0) and np.all(np.diff(got) <= 0)
    assert _orth_err(U) <= 1e-13
    # Nystrom is never worse than the direct method here, and the direct method obeys its bound
    Ud, gd = herm.direct_eig(A, Q, l)
    assert np.linalg.norm(E, 2) <= np.linalg.norm(A - (Ud * gd[None, :]) @ Ud.T, 2) * (1 + 1e-10)

