"""Pins of the single-pass oracle (oracle/single_pass.py), Algorithm 5.6 and the closing remark of
Section 5.5.

1. Exact case: a symmetric A of rank k (eigenvalues of both signs) with k + p Gaussian samples:
   Y spans range(A), the k leading left singular vectors of Y span it too, the system
   B (Q*Omega) = Q*Y is consistent with B = Q*AQ, and U Lambda U* = A with the prescribed
   eigenvalues in decreasing magnitude; also for p = 0 (square system, Q an orthonormal basis).
2. The least-squares core recovers a symmetric B0 exactly from N = B0 M for a rectangular k x (k+p)
   coefficient matrix M (a transposed or mis-oriented solve fails this).
3. The error bound behind the closing remark: with B_true = Q*AQ, Q*Y = B_true Q*Omega + E where
   E = Q*A(I - QQ*)Omega, so the least-squares B differs from B_true by at most
   ||E|| / sigma_min(Q*Omega), and ||A - U Lambda U*|| <= ||A - Q B_true Q*|| + ||E|| / sigma_min
   (checked on decaying spectra, with and without oversampling).
"""

import numpy as np
import pytest

from oracle import rsvd, single_pass
from workloads import build_symmetric


@pytest.mark.parametrize("p", [0, 4, 10])
def test_one_pass_exact_rank(p):
    n = 80
    lam = [3.0, -6.0, 1.5, -0.75, 0.5]
    k = len(lam)
    A = build_symmetric(n, lam, seed=71)
    Om = rsvd.gaussian_test_matrix(n, k + p, 72)
    U, got = single_pass.one_pass_eig(A, Om, k)
    expect = sorted(lam, key=lambda x: (-abs(x), -x))
    assert np.allclose(got, expect, rtol=0, atol=1e-11 * 6.0)
    assert np.linalg.norm(A - (U * got[None, :]) @ U.T, 2) <= 1e-11 * 6.0
    assert np.linalg.norm(U.T @ U - np.eye(k), 2) <= 1e-12


@pytest.mark.parametrize("k,p", [(6, 0), (6, 5), (12, 9)])
def test_core_recovers_symmetric_b(k, p):
    rng = np.random.default_rng(100 + k + p)
    B0 = rng.standard_normal((k, k))
    B0 = B0 + B0.T
    # Q = I_k, Omega = M, Y = N: the core sees M = Q*Omega and N = Q*Y
    M = rng.standard_normal((k, k + p))
    N = B0 @ M
    B = single_pass.least_squares_core(np.eye(k), M, N)
    assert np.linalg.norm(B - B0, 2) <= 1e-10 * np.linalg.norm(B0, 2)
    assert np.array_equal(B, B.T)


@pytest.mark.parametrize("decay,p,seed", [(1.0, 0, 81), (1.0, 8, 82), (2.0, 8, 83), (0.5, 16, 84)])
def test_one_pass_error_bound(decay, p, seed):
    n, k = 150, 10
    j = np.arange(1, n + 1, dtype=np.float64)
    lam = (-1.0) ** j * j ** -decay
    A = build_symmetric(n, lam, seed=seed)
    Om = rsvd.gaussian_test_matrix(n, k + p, seed + 1)
    Y = A @ Om
    Q = single_pass.one_pass_basis(Y, k)
    P = np.eye(n) - Q @ Q.T
    Btrue = Q.T @ A @ Q
    E = Q.T @ A @ P @ Om
    smin = np.linalg.svd(Q.T @ Om, compute_uv=False)[-1]
    U, got = single_pass.one_pass_eig(A, Om, k)
    err = np.linalg.norm(A - (U * got[None, :]) @ U.T, 2)
    err_true = np.linalg.norm(A - Q @ Btrue @ Q.T, 2)
    bound = err_true + np.linalg.norm(E, 2) / smin
    assert err <= bound * (1 + 1e-10), (err, err_true, bound)
    # and the core itself is within ||E|| / sigma_min of Q*AQ
    B = single_pass.least_squares_core(Q, Om, Y)
    assert np.linalg.norm(B - Btrue, 2) <= np.linalg.norm(E, 2) / smin * (1 + 1e-10)
