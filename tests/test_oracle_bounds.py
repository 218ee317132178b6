"""Pins of the oracle's error-bound formulas (Theorems 9.1, 10.5, 10.6, Corollaries 10.9, 10.10),
which the other tests only use as upper bounds -- a formula that is too loose would pass there.

1. Values evaluated by hand from the theorem statements at the workloads' spectra, independently of
   this code (3 significant digits): for sigma_j = e^{-j/20}, n = 1000, k = 20, p = 10, Theorem 10.6
   gives 7.32 sigma_21 (sigma_21 = 0.34994), Corollary 10.9 gives 43.4 sigma_21 (form with failure
   probability 6 e^-p) and 264.5 sigma_21 (form with 6 p^-p), Theorem 10.5 gives 2.036 with the
   optimal Frobenius error 1.1344; for sigma_j = 1/j, n = 8192, k = 100, p = 20, Corollary 10.10
   gives 18.2, 2.16, 1.53 sigma_101 at q = 0, 1, 2; for sigma_j = j^-1/2, n = 2048, k = 64, p = 16,
   q = 1 it gives 2.28 sigma_65.
2. Structure: Corollary 10.10 is Theorem 10.6 applied to (A A*)^q A, so at q = 0 the two coincide.
3. Closed forms the bounds are built from (Propositions 10.1 and 10.2): for a standard Gaussian
   k x (k + p) matrix G, E ||G^+||_F^2 = k / (p - 1), so E ||Sigma_2 Omega_2 Omega_1^+||_F^2 =
   k / (p - 1) ||Sigma_2||_F^2, and the square of the Theorem 10.5 bound equals ||Sigma_2||_F^2 plus
   that expectation.  Checked by Monte Carlo.
4. Theorem 9.1 is attained when the test matrix spans the top right singular space (Omega_2 = 0):
   the bound is then exactly sigma_(k+1), which is also the error.
"""

import numpy as np

from oracle import evaluate


def test_bounds_match_hand_evaluated_values():
    j = np.arange(1, 1001)
    s = np.exp(-j / 20.0)
    s21 = s[20]
    assert abs(s21 - 0.34994) < 1e-5
    assert round(evaluate.thm10_6_bound(s, 20, 10) / s21, 2) == 7.32
    assert round(evaluate.cor10_9_bound(s, 20, 10, form=1) / s21, 1) == 43.4
    assert round(evaluate.cor10_9_bound(s, 20, 10, form=2) / s21, 1) == 264.5
    assert round(evaluate.thm10_5_bound(s, 20, 10), 3) == 2.036
    assert round(float(np.sqrt(np.sum(s[20:] ** 2))), 4) == 1.1344
    s = 1.0 / np.arange(1, 8193)
    assert [round(evaluate.cor10_10_bound(s, 100, 20, q) / s[100], 2) for q in (0, 1, 2)] == [18.20, 2.16, 1.53]
    s = np.arange(1, 2049) ** -0.5
    assert round(evaluate.cor10_10_bound(s, 64, 16, 1) / s[64], 2) == 2.28


def test_cor10_10_at_q0_is_thm10_6():
    rng = np.random.default_rng(3)
    for _ in range(5):
        s = np.sort(rng.exponential(size=300))[::-1]
        k, p = int(rng.integers(2, 40)), int(rng.integers(2, 20))
        a, b = evaluate.cor10_10_bound(s, k, p, 0), evaluate.thm10_6_bound(s, k, p)
        assert abs(a - b) <= 1e-14 * b


def test_thm10_5_is_built_from_the_gaussian_pseudoinverse_expectation():
    # E ||G^+||_F^2 = k / (p - 1) for G standard Gaussian k x (k + p) (Proposition 10.2), hence
    # E ||Sigma_2 Omega_2 Omega_1^+||_F^2 = k / (p - 1) ||Sigma_2||_F^2 (Proposition 10.1) and the
    # Theorem 10.5 bound squared is ||Sigma_2||_F^2 (1 + k / (p - 1)).
    rng = np.random.default_rng(11)
    k, p, tail = 6, 5, 40
    s2 = np.linspace(1.0, 0.2, tail)
    samples = []
    for _ in range(4000):
        O1 = rng.standard_normal((k, k + p))
        O2 = rng.standard_normal((tail, k + p))
        samples.append(np.linalg.norm((s2[:, None] * O2) @ np.linalg.pinv(O1), "fro") ** 2)
    mc = float(np.mean(samples))
    exact = k / (p - 1.0) * float(np.sum(s2 ** 2))
    se = float(np.std(samples)) / np.sqrt(len(samples))
    assert abs(mc - exact) <= 4 * se, (mc, exact, se)
    sigma = np.r_[np.full(k, 2.0), s2]
    assert abs(evaluate.thm10_5_bound(sigma, k, p) ** 2 - (np.sum(s2 ** 2) + exact)) <= 1e-12 * exact


def test_thm9_1_attained_when_omega_spans_top_right_space():
    rng = np.random.default_rng(2)
    n, k, p = 40, 5, 3
    V = np.linalg.qr(rng.standard_normal((n, n)))[0]
    sigma = np.sort(rng.uniform(0.1, 3.0, n))[::-1]
    Omega = V[:, :k] @ rng.standard_normal((k, k + p))  # Omega_2 = V_2* Omega = 0
    assert abs(evaluate.thm9_1_bound(sigma, V, Omega, k) - sigma[k]) <= 1e-12 * sigma[k]
    U = np.linalg.qr(rng.standard_normal((60, n)))[0]
    A = (U * sigma) @ V.T
    Q = np.linalg.qr(A @ Omega)[0][:, :k]  # range(A Omega) has dimension k
    assert abs(evaluate.residual_q(A, Q) - sigma[k]) <= 1e-10 * sigma[k]
