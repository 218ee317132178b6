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
4. The two-sided single pass for a general A: the core recovers B exactly from two consistent
   rectangular relations; a rank-r A is factored exactly from l >= r samples on each side; and the
   least-squares B is within ||(E1, E2)||_F / sqrt(sigma_min(M1)^2 + sigma_min(M2)^2) of Q*A Qt
   (Frobenius), E1, E2 the residuals of the two relations at Q*A Qt.
5. The normal-equation route to the same core (for large l) agrees with the stacked least-squares
   solve on well-conditioned relations, and recovers B exactly from consistent ones.
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


# --- the two-sided single pass for a general A (Section 5.5) -------------------------------------

@pytest.mark.parametrize("l,lt,s1,s2", [(5, 4, 6, 7), (6, 6, 6, 6), (3, 5, 8, 4)])
def test_two_sided_core_recovers_b(l, lt, s1, s2):
    # consistent relations B M1 = N1, B^T M2 = N2 with full-rank M1 (lt x s1), M2 (l x s2): B exactly
    rng = np.random.default_rng(200 + l + lt)
    B0 = rng.standard_normal((l, lt))
    M1 = rng.standard_normal((lt, s1))
    M2 = rng.standard_normal((l, s2))
    B = single_pass.two_sided_core(M1, B0 @ M1, M2, B0.T @ M2)
    assert np.linalg.norm(B - B0) <= 1e-10 * np.linalg.norm(B0)


@pytest.mark.parametrize("m,n,r,l", [(90, 60, 5, 8), (70, 110, 6, 6)])
def test_two_sided_exact_rank(m, n, r, l):
    from workloads import build_matrix
    sigma = np.zeros(min(m, n))
    sigma[:r] = np.linspace(3.0, 0.5, r)
    A = build_matrix(m, n, sigma, seed=101)
    Om = rsvd.gaussian_test_matrix(n, l, 102, 0)
    Omt = rsvd.gaussian_test_matrix(m, l, 102, 1)
    U, S, V = single_pass.two_sided_svd(A, Om, Omt, r)
    assert np.allclose(S, sigma[:r], rtol=1e-10, atol=0)
    assert np.linalg.norm(A - (U * S[None, :]) @ V.T, 2) <= 1e-10 * 3.0
    assert np.linalg.norm(U.T @ U - np.eye(r), 2) <= 1e-12
    assert np.linalg.norm(V.T @ V - np.eye(r), 2) <= 1e-12


@pytest.mark.parametrize("decay,seed", [(1.0, 111), (2.0, 112)])
def test_two_sided_core_error_bound(decay, seed):
    # N1 = B_true M1 + E1, N2 = B_true^T M2 + E2 with B_true = Q*A Qt: the least-squares B is within
    # ||(E1, E2)||_F / sqrt(sigma_min(M1)^2 + sigma_min(M2)^2) of B_true (Frobenius)
    from workloads import build_matrix
    m, n, l = 120, 90, 10
    sigma = np.arange(1, 91, dtype=np.float64) ** -decay
    A = build_matrix(m, n, sigma, seed=seed)
    Om = rsvd.gaussian_test_matrix(n, l, seed + 1, 0)
    Omt = rsvd.gaussian_test_matrix(m, l, seed + 1, 1)
    Q, _ = rsvd.qr_pos(A @ Om)
    Qt, _ = rsvd.qr_pos(A.T @ Omt)
    M1, M2 = Qt.T @ Om, Q.T @ Omt
    N1, N2 = Q.T @ A @ Om, Qt.T @ A.T @ Omt
    Bt = Q.T @ A @ Qt
    E1, E2 = N1 - Bt @ M1, N2 - Bt.T @ M2
    s1 = np.linalg.svd(M1, compute_uv=False)[-1]
    s2 = np.linalg.svd(M2, compute_uv=False)[-1]
    bound = np.sqrt(np.linalg.norm(E1) ** 2 + np.linalg.norm(E2) ** 2) / np.sqrt(s1 ** 2 + s2 ** 2)
    B = single_pass.two_sided_core(M1, N1, M2, N2)
    assert np.linalg.norm(B - Bt) <= bound * (1 + 1e-10), (np.linalg.norm(B - Bt), bound)


@pytest.mark.parametrize("l,lt,s1,s2,consistent", [(5, 4, 6, 7, True), (8, 8, 8, 8, False), (6, 9, 12, 7, False)])
def test_two_sided_normal_route_matches_lstsq(l, lt, s1, s2, consistent):
    rng = np.random.default_rng(300 + l + lt)
    B0 = rng.standard_normal((l, lt))
    M1 = rng.standard_normal((lt, s1))
    M2 = rng.standard_normal((l, s2))
    N1 = B0 @ M1 + (0.0 if consistent else 0.1 * rng.standard_normal((l, s1)))
    N2 = B0.T @ M2 + (0.0 if consistent else 0.1 * rng.standard_normal((lt, s2)))
    Bn = single_pass.two_sided_core_normal(M1, N1, M2, N2)
    Bl = single_pass.two_sided_core(M1, N1, M2, N2)
    assert np.linalg.norm(Bn - Bl) <= 1e-10 * np.linalg.norm(Bl)
    if consistent:
        assert np.linalg.norm(Bn - B0) <= 1e-10 * np.linalg.norm(B0)
