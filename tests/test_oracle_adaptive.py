"""Pins of the fixed-precision range finder's oracle (oracle/adaptive.py), Sections 4.3-4.4.

1. The a posteriori estimate, eq. (4.3) and the lemma after it: for a rank-one B the failure event
   ||B|| > 10 sqrt(2/pi) ||B w|| is |g| < 1/(10 sqrt(2/pi)) for one standard normal g, probability
   2 Phi(0.1253) - 1 = 0.0998 <= 10^-1: a sharp check of the constant (r = 1), and of the union over
   r = 2 vectors (probability 0.0998^2 <= 10^-2).
2. Algorithm 4.2 on a matrix of exact rank k stops with j = k: after k samples every projected
   sample is at roundoff level, and before that none is (the r-window test cannot pass early on a
   generic matrix with sigma_k far above eps).
3. Algorithm 4.2 meets its tolerance: ||(I - Q Q*) A|| <= eps on every one of 40 seeds (failure
   probability at most min(m, n) 10^-r with r = 10), and Q is orthonormal; its basis is never
   smaller than the Mirsky bound allows (sigma_(j+1) <= ||(I - QQ*) A||).
4. The blocked form: on an exact-rank matrix it returns the first basis size of its doubling
   schedule that is >= the rank, spanning range(A); on decaying spectra the returned basis meets
   eps, every earlier test block failed (its estimate > eps), and the accepted estimate bounds the
   true error.
"""

import math

import numpy as np
import pytest

from oracle import adaptive, evaluate, philox
from workloads import build_matrix, spectrum


def test_estimate_constant_rank_one():
    rng = np.random.default_rng(0)
    u = rng.standard_normal(40)
    v = rng.standard_normal(30)
    B = np.outer(u, v)
    nB = np.linalg.norm(B, 2)
    trials = 40000
    W = rng.standard_normal((30, trials))
    ratio = np.linalg.norm(B @ W, axis=0) * adaptive.errorest_factor()
    p1 = float(np.mean(nB > ratio))
    expect = math.erf(1.0 / adaptive.errorest_factor() / math.sqrt(2.0))  # P(|g| < 1 / factor)
    assert abs(expect - 0.0998) < 5e-4 and expect <= 0.1
    assert abs(p1 - expect) <= 4 * math.sqrt(expect * (1 - expect) / trials), (p1, expect)
    pairs = np.maximum(ratio[0::2], ratio[1::2])
    p2 = float(np.mean(nB > pairs))
    assert p2 <= 0.01 + 4 * math.sqrt(0.01 * 0.99 / pairs.size), p2
    # the helper evaluates the same right-hand side
    assert abs(adaptive.posterior_estimate(B, W[:, :3]) - np.max(ratio[:3])) <= 1e-12 * nB


@pytest.mark.parametrize("k", [3, 11, 25])
def test_alg42_exact_rank_stops_at_rank(k):
    m, n, r = 120, 80, 10
    sigma = np.zeros(n)
    sigma[:k] = np.linspace(2.0, 0.5, k)
    A = build_matrix(m, n, sigma, seed=k)
    Om = philox.gaussian_omega(n, n + r, seed=5, stream=k)
    Q, j = adaptive.adaptive_range_finder(A, 1e-8, r, Om)
    assert j == k
    assert evaluate.residual_q(A, Q) <= 1e-12
    assert evaluate.orthonormality_error(Q) <= 1e-13


def test_alg42_meets_tolerance():
    m, n, r, eps = 200, 120, 10, 1e-3
    sigma = spectrum("exp_r", n, rate=6.0)
    A = build_matrix(m, n, sigma, seed=4)
    for seed in range(40):
        Om = philox.gaussian_omega(n, n + r, seed=seed + 100, stream=0)
        Q, j = adaptive.adaptive_range_finder(A, eps, r, Om)
        err = evaluate.residual_q(A, Q)
        assert err <= eps, (seed, err)
        assert sigma[j] <= err * (1 + 1e-10)  # Mirsky: no j-column basis does better than sigma_(j+1)
        assert evaluate.orthonormality_error(Q) <= 1e-12


@pytest.mark.parametrize("rank,b0,lmax,expect", [(5, 8, 64, 8), (9, 8, 64, 16), (17, 8, 64, 32),
                                                 (33, 8, 64, 64), (12, 12, 48, 12)])
def test_blocked_exact_rank(rank, b0, lmax, expect):
    m, n, r = 150, 100, 8
    sigma = np.zeros(n)
    sigma[:rank] = np.linspace(3.0, 1.0, rank)
    A = build_matrix(m, n, sigma, seed=rank)
    Om = philox.gaussian_omega(n, lmax + r, seed=9, stream=rank)
    out = adaptive.blocked_adaptive_range_finder(A, 1e-7, r, b0, lmax, Om)
    assert out["l"] == expect and out["converged"]
    assert evaluate.residual_q(A, out["Q"]) <= 1e-12
    assert evaluate.orthonormality_error(out["Q"]) <= 1e-12
    assert adaptive.block_schedule(b0, lmax)[: len(out["tested"])][-1] <= lmax


@pytest.mark.parametrize("eps", [3e-2, 1e-3, 1e-4])
def test_blocked_meets_tolerance(eps):
    m, n, r, b0, lmax = 300, 200, 10, 16, 128
    sigma = spectrum("exp_r", n, rate=8.0)
    A = build_matrix(m, n, sigma, seed=7)
    for seed in range(20):
        Om = philox.gaussian_omega(n, lmax + r, seed=seed, stream=1)
        out = adaptive.blocked_adaptive_range_finder(A, eps, r, b0, lmax, Om)
        err = evaluate.residual_q(A, out["Q"])
        assert out["converged"]
        assert err <= eps and err <= out["est"], (seed, err, out["est"])
        assert all(e > eps for e in out["tested"][:-1])
        assert out["l"] in (0, 16, 32, 64, 128)
        assert sigma[out["l"]] <= err * (1 + 1e-10)


def test_blocked_capacity_not_converged():
    # a flat spectrum that no 32-column basis captures to 1e-6: the range finder stops at lmax and
    # reports the last estimate, which bounds the true error
    m, n, r, b0, lmax = 200, 150, 6, 8, 32
    sigma = np.linspace(1.0, 0.5, n)
    A = build_matrix(m, n, sigma, seed=3)
    Om = philox.gaussian_omega(n, lmax + r, seed=2)
    out = adaptive.blocked_adaptive_range_finder(A, 1e-6, r, b0, lmax, Om)
    assert out["l"] == lmax and not out["converged"]
    assert evaluate.residual_q(A, out["Q"]) <= out["est"]
    assert len(out["tested"]) == len(adaptive.block_schedule(b0, lmax)) + 1
