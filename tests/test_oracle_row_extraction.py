"""Pins of the row-extraction oracle (oracle/row_extraction.py; Algorithm 5.2, Section 5.2).

1. The ID reproduces its matrix: B = X B(J,:) to rounding, X(J,:) = I exactly, J has k distinct
   indices; on a matrix whose first k rows are the identity (J = those rows is an exact ID with X = B)
   the ID recovers B from any J it picks.
2. Exact rank: when range(A) lies in range(Q), A = X A(J,:) exactly, so Algorithm 5.2 reproduces A
   (up to rounding) and its singular values are A's.
3. The bound of the lemma's proof, ||A - U S V*|| <= (1 + ||X||) ||A - Q Q* A||, on decaying spectra
   with Q from the range finder, for the ID of Q and of the sample matrix Y (the remark after the
   algorithm); and the stated bound [1 + sqrt(1 + 4k(m - k))] eps whenever max |X| <= 2.
4. The outputs are an SVD: U and V orthonormal, S nonnegative and descending.
"""

import numpy as np
import pytest

from oracle import row_extraction as rx, rsvd
from workloads import build_matrix


@pytest.mark.parametrize("m,k,seed", [(40, 5, 1), (200, 20, 2), (64, 64, 3)])
def test_row_id_reproduces(m, k, seed):
    B = np.random.default_rng(seed).standard_normal((m, k))
    J, X = rx.row_id(B)
    assert len(set(J.tolist())) == k
    assert np.array_equal(X[J, :], np.eye(k))
    assert np.linalg.norm(B - X @ B[J, :]) <= 1e-12 * np.linalg.norm(B)


def test_row_id_of_identity_block():
    rng = np.random.default_rng(4)
    k = 6
    B = np.vstack([np.eye(k), 0.3 * rng.standard_normal((30, k))])
    J, X = rx.row_id(B)
    assert np.linalg.norm(B - X @ B[J, :]) <= 1e-13


@pytest.mark.parametrize("m,n,r,l", [(120, 80, 6, 6), (90, 150, 8, 10)])
def test_exact_rank_reproduces_a(m, n, r, l):
    sigma = np.zeros(min(m, n))
    sigma[:r] = np.linspace(4.0, 0.5, r)
    A = build_matrix(m, n, sigma, seed=10 + r)
    Q = rsvd.randomized_range_finder(A, rsvd.gaussian_test_matrix(n, l, 11))
    U, S, V, J, X = rx.extract_rows_svd(A, Q)
    assert np.linalg.norm(A - (U * S[None, :]) @ V.T, 2) <= 1e-10 * 4.0
    assert np.allclose(S[:r], sigma[:r], rtol=1e-9, atol=0)


@pytest.mark.parametrize("decay,use_y,seed", [(1.0, False, 21), (2.0, False, 22), (1.0, True, 23), (0.5, True, 24)])
def test_error_bound(decay, use_y, seed):
    m, n, k = 150, 100, 12
    sigma = np.arange(1, 101, dtype=np.float64) ** -decay
    A = build_matrix(m, n, sigma, seed=seed)
    Om = rsvd.gaussian_test_matrix(n, k, seed + 1)
    Y = A @ Om
    Q, _ = rsvd.qr_pos(Y)
    eps = np.linalg.norm(A - Q @ (Q.T @ A), 2)
    U, S, V, J, X = rx.extract_rows_svd(A, Y if use_y else Q)
    err = np.linalg.norm(A - (U * S[None, :]) @ V.T, 2)
    assert err <= (1 + np.linalg.norm(X, 2)) * eps * (1 + 1e-9), (err, eps, np.linalg.norm(X, 2))
    if np.max(np.abs(X)) <= 2.0:
        assert err <= (1 + np.sqrt(1 + 4 * k * (m - k))) * eps
    assert np.linalg.norm(U.T @ U - np.eye(k), 2) <= 1e-12
    assert np.linalg.norm(V.T @ V - np.eye(k), 2) <= 1e-12
    assert np.all(S >= 0) and np.all(np.diff(S) <= 0)
