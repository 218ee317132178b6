"""Pins for the oracle's randomized SVD (CPU only).

Nothing here compares the oracle with itself.  Each test checks it against a
fact the paper or plain mathematics fixes:
  * brute force: with l = min(m, n) the range finder captures all of range(A),
    so the result must be LAPACK's full SVD of A;
  * exact recovery of an exact-rank matrix (Section 1.3, Theorem 9.1 with
    Sigma2 = 0);
  * the deterministic bounds of Section 9 for the very Omega drawn
    (Theorems 9.1, 9.2, 9.3) and the Mirsky lower bound;
  * the "no worse" identity of Algorithm 5.1: the untruncated U S V* equals
    QQ*A;
  * Algorithm 4.4 spans the same space as Algorithm 4.3 (exact arithmetic);
  * the SRFT sketch equals A times the SRFT matrix written out from its
    definition with an O(n^2) DFT;
  * averages over seeds stay under Theorem 10.6 and Corollary 10.10.
"""

import numpy as np
import pytest

from oracle import evaluate, philox, rsvd
from workloads import build_matrix, spectrum


def _matrix(m, n, sigma, seed=7):
    A, U, V = build_matrix(m, n, sigma, seed=seed, return_factors=True)
    return A, U, V


def test_qr_pos_is_a_qr():
    rng = np.random.default_rng(0)
    for shape in [(30, 7), (9, 9), (50, 1)]:
        Y = rng.standard_normal(shape)
        Q, R = rsvd.qr_pos(Y)
        assert np.allclose(Q @ R, Y, atol=1e-13)
        assert evaluate.orthonormality_error(Q) < 1e-14
        assert np.allclose(np.tril(R, -1), 0)
        assert np.all(np.diag(R) > 0)


def test_qr_pos_equals_gram_schmidt():
    # For full-rank Y the QR with positive diag(R) is unique: classical
    # Gram-Schmidt written out column by column must give the same Q.
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((12, 5))
    Qgs = np.zeros_like(Y)
    for j in range(5):
        v = Y[:, j].copy()
        for i in range(j):
            v -= (Qgs[:, i] @ Y[:, j]) * Qgs[:, i]
        Qgs[:, j] = v / np.linalg.norm(v)
    Q, _ = rsvd.qr_pos(Y)
    assert np.allclose(Q, Qgs, atol=1e-12)


def test_qr_pos_complex():
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((20, 6)) + 1j * rng.standard_normal((20, 6))
    Q, R = rsvd.qr_pos(Y)
    assert np.allclose(Q @ R, Y, atol=1e-13)
    assert np.allclose(np.imag(np.diag(R)), 0) and np.all(np.real(np.diag(R)) > 0)


@pytest.mark.parametrize("m,n,q", [(12, 8, 0), (40, 25, 0), (40, 25, 2), (25, 25, 1)])
def test_full_sample_count_gives_exact_svd(m, n, q):
    # l = min(m, n): range(Y) = range(A), so Stage B returns the SVD of A.
    sigma = spectrum("exp_r", min(m, n), rate=4.0)
    A, _, _ = _matrix(m, n, sigma)
    r = min(m, n)
    k = r - 2
    out = rsvd.rsvd(A, k, 2, q, seed=3)
    U0, S0, Vh0 = np.linalg.svd(A, full_matrices=False)
    np.testing.assert_allclose(out["S"], S0, rtol=1e-10, atol=1e-14)
    Uk, Vk = rsvd.normalize_signs(out["Uk"], out["Vk"])
    Ur, Vr = rsvd.normalize_signs(U0[:, :k], Vh0[:k].T)
    assert np.max(np.abs(Uk - Ur)) < 1e-9
    assert np.max(np.abs(Vk - Vr)) < 1e-9


@pytest.mark.parametrize("q", [0, 1])
def test_exact_rank_recovery(q):
    # A of exact rank 6 < l: the samples span range(A) (Theorem 9.1 with Sigma2 = 0).
    m, n, rank = 80, 50, 6
    sigma = np.zeros(50)
    sigma[:rank] = [5.0, 3.0, 2.0, 1.0, 0.5, 0.25]
    A, _, _ = _matrix(m, n, sigma)
    out = rsvd.rsvd(A, rank, 4, q, seed=11)
    np.testing.assert_allclose(out["Sk"], sigma[:rank], rtol=1e-12)
    assert evaluate.residual_q(A, out["Q"]) < 1e-13 * sigma[0]
    assert evaluate.residual_usv(A, out["Uk"], out["Sk"], out["Vk"]) < 1e-13 * sigma[0]


def test_deterministic_bounds_section_9():
    m, n, k, p = 300, 200, 10, 5
    sigma = spectrum("exp_r", n, rate=6.0)
    A, U, V = _matrix(m, n, sigma)
    for seed in range(5):
        out = rsvd.rsvd(A, k, p, 0, seed=seed)
        res_q = evaluate.residual_q(A, out["Q"])
        res_k = evaluate.residual_usv(A, out["Uk"], out["Sk"], out["Vk"])
        res_full = evaluate.residual_usv(A, out["U"], out["S"], out["V"])
        l = k + p
        # Mirsky: no rank-l matrix does better than sigma_{l+1}
        assert res_q >= sigma[l] * (1 - 1e-10)
        assert res_k >= sigma[k] * (1 - 1e-10)
        # Theorem 9.1 for this Omega
        assert res_q <= evaluate.thm9_1_bound(sigma, V, out["Omega"], k) * (1 + 1e-10)
        # Algorithm 5.1 does not degrade the error: U S V* = QQ*A exactly
        assert abs(res_full - res_q) <= 1e-12 * sigma[0]
        # Theorem 9.3 for the truncated factorization
        assert res_k <= evaluate.thm9_3_bound(sigma, k, res_q) * (1 + 1e-10)
        # interlacing: singular values of Q*A never exceed those of A
        assert np.all(out["S"] <= sigma[:l] * (1 + 1e-12))


@pytest.mark.parametrize("q", [1, 2])
def test_power_scheme_theorem_9_2(q):
    m, n, k, p = 200, 150, 8, 4
    sigma = spectrum("inv", n)
    A, _, _ = _matrix(m, n, sigma)
    Om = rsvd.gaussian_test_matrix(n, k + p, seed=4)
    Qz = rsvd.randomized_subspace_iteration(A, Om, q)
    Bq = A.copy()
    for _ in range(q):
        Bq = A @ (A.T @ Bq)
    lhs = evaluate.residual_q(A, Qz)
    rhs = evaluate.residual_q(Bq, Qz) ** (1.0 / (2 * q + 1))
    assert lhs <= rhs * (1 + 1e-8)
    # and the power scheme helps on a slowly decaying spectrum
    Q0 = rsvd.randomized_range_finder(A, Om)
    assert lhs < evaluate.residual_q(A, Q0)


@pytest.mark.parametrize("m,n", [(120, 90), (90, 90)])
def test_subspace_iteration_spans_power_iteration(m, n):
    # Remark 4.3: Algorithms 4.3 and 4.4 agree in exact arithmetic; on a mildly
    # conditioned problem their projectors agree to rounding.
    k, p, q = 6, 4, 1
    sigma = np.linspace(2.0, 1.0, n)
    A, _, _ = _matrix(m, n, sigma)
    Om = rsvd.gaussian_test_matrix(n, k + p, seed=8)
    Q3 = rsvd.randomized_power_iteration(A, Om, q)
    Q4 = rsvd.randomized_subspace_iteration(A, Om, q)
    assert np.max(np.abs(Q3 @ Q3.T - Q4 @ Q4.T)) < 1e-10


def test_srft_sketch_equals_definition():
    rng = np.random.default_rng(5)
    m, n, l = 7, 24, 6
    A = rng.standard_normal((m, n))
    d = philox.srft_signs(n, seed=1)
    R = philox.srft_sample(n, l, seed=1)
    Om = rsvd.srft_test_matrix(n, d, R)
    np.testing.assert_allclose(rsvd.srft_sketch(A, d, R), A @ Om, atol=1e-12)
    # F is unitary, so the full (unsampled) SRFT with l = n is sqrt(n/l) times unitary
    Rall = np.arange(n)
    Ofull = rsvd.srft_test_matrix(n, d, Rall)
    np.testing.assert_allclose(Ofull.conj().T @ Ofull, np.eye(n), atol=1e-12)


def test_real_fourier_basis_is_the_dft_mixed_in_pairs():
    # F_r = F T with F the unitary DFT of Section 4.6 and T unitary, pairing
    # frequencies q and n - q: the real basis spans the same frequencies.
    n = 16
    p = np.arange(n)[:, None]
    F = np.exp(-2j * np.pi * p * np.arange(n)[None, :] / n) / np.sqrt(n)
    T = np.zeros((n, n), dtype=complex)
    T[0, 0] = 1.0
    T[n // 2, n // 2] = 1.0
    for q in range(1, n // 2):
        T[q, q] = T[n - q, q] = 1 / np.sqrt(2)            # cosine column
        T[q, n - q], T[n - q, n - q] = 1j / np.sqrt(2), -1j / np.sqrt(2)  # sine column
    assert np.allclose(T.conj().T @ T, np.eye(n))
    Fr = rsvd.real_fourier_matrix(n)
    np.testing.assert_allclose(F @ T, Fr, atol=1e-13)
    np.testing.assert_allclose(Fr.T @ Fr, np.eye(n), atol=1e-13)


@pytest.mark.parametrize("n,l", [(32, 6), (64, 64), (16, 3)])
def test_real_srft_sketch_equals_definition(n, l):
    rng = np.random.default_rng(n + l)
    A = rng.standard_normal((9, n))
    d = philox.srft_signs(n, seed=4)
    R = philox.srft_sample(n, l, seed=4)
    np.testing.assert_allclose(rsvd.real_srft_sketch(A, d, R), A @ rsvd.real_srft_test_matrix(n, d, R),
                               atol=1e-12)


def test_real_srft_full_sample_is_orthogonal_mixing():
    # l = n: Omega = D F_r is orthogonal, so Y = A Omega preserves all singular values
    n = 32
    A = np.random.default_rng(3).standard_normal((40, n))
    d = philox.srft_signs(n, seed=1)
    R = philox.srft_sample(n, n, seed=1)
    Y = rsvd.real_srft_sketch(A, d, R)
    np.testing.assert_allclose(np.linalg.svd(Y, compute_uv=False), np.linalg.svd(A, compute_uv=False),
                               rtol=1e-12)


@pytest.mark.parametrize("sketch", ["srft", "srft_complex"])
def test_srft_pipeline_exact_rank(sketch):
    m, n, rank = 64, 32, 5
    sigma = np.zeros(32)
    sigma[:rank] = [4, 3, 2, 1, 0.5]
    A, _, _ = _matrix(m, n, sigma)
    out = rsvd.rsvd(A, rank, 7, 0, seed=2, sketch=sketch)
    np.testing.assert_allclose(out["Sk"], sigma[:rank], rtol=1e-12)
    assert np.iscomplexobj(out["Q"]) == (sketch == "srft_complex")
    assert evaluate.residual_q(A, out["Q"]) < 1e-12
    assert evaluate.orthonormality_error(out["Q"]) < 1e-13


def test_average_error_under_theorem_10_6():
    m, n, k, p = 200, 100, 10, 5
    sigma = spectrum("exp_r", n, rate=8.0)
    A, _, _ = _matrix(m, n, sigma)
    errs = [evaluate.residual_q(A, rsvd.rsvd(A, k, p, 0, seed=s)["Q"]) for s in range(60)]
    assert np.mean(errs) <= evaluate.thm10_6_bound(sigma, k, p)
    # the per-instance deviation bound of Corollary 10.9 (failure prob <= 6 e^-5)
    assert max(errs) <= evaluate.cor10_9_bound(sigma, k, p, form=1)


def test_average_error_under_corollary_10_10():
    m, n, k, p, q = 200, 100, 10, 5, 1
    sigma = spectrum("inv", n)
    A, _, _ = _matrix(m, n, sigma)
    errs = [evaluate.residual_q(A, rsvd.rsvd(A, k, p, q, seed=s)["Q"]) for s in range(40)]
    assert np.mean(errs) <= evaluate.cor10_10_bound(sigma, k, p, q)


def test_operator_norm_path_matches_dense():
    m, n = 300, 120
    sigma = spectrum("inv", n)
    A, _, _ = _matrix(m, n, sigma)
    out = rsvd.rsvd(A, 10, 5, 1, seed=0)
    dense = evaluate.residual_q(A, out["Q"])
    old = evaluate.DENSE_LIMIT
    try:
        evaluate.DENSE_LIMIT = 0
        op = evaluate.residual_q(A, out["Q"])
        op_k = evaluate.residual_usv(A, out["Uk"], out["Sk"], out["Vk"])
    finally:
        evaluate.DENSE_LIMIT = old
    assert abs(op - dense) <= 1e-9 * dense
    assert abs(op_k - evaluate.residual_usv(A, out["Uk"], out["Sk"], out["Vk"])) <= 1e-9 * op_k


def test_input_dtype_rounding_is_respected():
    # FP32 configs feed the oracle float64(float32(A)); Omega is rounded the same way.
    Om32 = rsvd.gaussian_test_matrix(10, 6, seed=1, dtype=np.float32)
    Om64 = rsvd.gaussian_test_matrix(10, 6, seed=1)
    assert np.array_equal(Om32, Om64.astype(np.float32).astype(np.float64))
    assert not np.array_equal(Om32, Om64)
