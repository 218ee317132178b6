"""Pins of the Givens-chain test matrix oracle (oracle/gsrft.py; the remark on random Givens rotations
in Section 4.6, real form).

1. A chain applied to e_1 has the closed form (x G_1 ... G_{n-1})_j = c_j prod_{i<j} s_i (j < n - 1),
   prod_i s_i (j = n - 1); applied to e_{n-1} only the last rotation acts.  A sign or index slip in
   the rotation formulas, or rotations applied in the wrong order, fails one of these.
2. The row-by-row application of D Theta equals the row vector times the dense product
   D Pi G(1,2) ... G(n-1,n) built from the definitions (the permutation as a matrix with
   Pi_ij = 1 for i = pi(j), each G as a full rotation matrix).
3. The factors are orthogonal: the pretransform T = D'' Theta' D' Theta satisfies T T^T = I, and
   the dense Omega satisfies Omega^T Omega = (n/l) I (T D F_r orthogonal, R distinct columns).
4. The sketch through the factored form equals A times the dense Omega.
5. The permutations are permutations, their distribution is uniform (chi-square over seeds), and the
   angles are uniform on [0, 2 pi) (mean of cos and sin near 0).
6. With l >= rank(A) samples the range finder captures range(A) exactly.
"""

import numpy as np
import pytest

from oracle import gsrft, philox, rsvd


def test_chain_closed_form():
    n = 9
    theta = philox.givens_angles(n, 11, 0)
    c, s = np.cos(theta), np.sin(theta)
    e1 = np.zeros((1, n))
    e1[0, 0] = 1.0
    y = gsrft.rotation_chain_rows(e1, theta)[0]
    expect = np.array([c[j] * np.prod(s[:j]) for j in range(n - 1)] + [np.prod(s)])
    assert np.allclose(y, expect, rtol=0, atol=1e-15)
    en = np.zeros((1, n))
    en[0, -1] = 1.0
    y = gsrft.rotation_chain_rows(en, theta)[0]
    expect = np.zeros(n)
    expect[-2], expect[-1] = -s[-1], c[-1]
    assert np.allclose(y, expect, rtol=0, atol=1e-15)


def _dense_factor(d, pi, theta):
    n = d.size
    M = np.diag(d)
    P = np.zeros((n, n))
    P[pi, np.arange(n)] = 1.0  # Pi_ij = 1 for i = pi(j)
    M = M @ P
    for j, th in enumerate(theta):
        G = np.eye(n)
        G[j, j] = G[j + 1, j + 1] = np.cos(th)
        G[j, j + 1] = np.sin(th)
        G[j + 1, j] = -np.sin(th)
        M = M @ G
    return M


@pytest.mark.parametrize("n,seed", [(8, 3), (16, 4), (32, 5)])
def test_factor_matches_dense_product(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((5, n))
    for chain in (0, 1):
        d = philox.givens_signs(n, seed, chain)
        pi = philox.givens_permutation(n, seed, chain)
        theta = philox.givens_angles(n, seed, chain)
        got = gsrft.givens_factor_rows(X, d, pi, theta)
        assert np.allclose(got, X @ _dense_factor(d, pi, theta), rtol=0, atol=1e-13)
    (d0, p0, t0), (d1, p1, t1) = gsrft.draws(n, seed)
    T = _dense_factor(d1, p1, t1) @ _dense_factor(d0, p0, t0)
    assert np.allclose(gsrft.pretransform_rows(X, seed), X @ T, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n,l,seed", [(16, 6, 7), (64, 20, 8)])
def test_orthogonality(n, l, seed):
    T = gsrft.pretransform_rows(np.eye(n), seed)
    assert np.linalg.norm(T @ T.T - np.eye(n), 2) <= 1e-13
    Om = gsrft.gsrft_test_matrix(n, l, seed)
    assert np.linalg.norm(Om.T @ Om - (n / l) * np.eye(l), 2) <= 1e-12 * n / l


@pytest.mark.parametrize("m,n,l,seed", [(12, 16, 5, 9), (30, 64, 17, 10)])
def test_sketch_matches_dense(m, n, l, seed):
    A = np.random.default_rng(seed).standard_normal((m, n))
    Y = gsrft.gsrft_sketch(A, l, seed)
    assert np.allclose(Y, A @ gsrft.gsrft_test_matrix(n, l, seed), rtol=0, atol=1e-12)


def test_permutation_uniform_and_angles_uniform():
    n, trials = 6, 3000
    counts = np.zeros((n, n))
    for seed in range(trials):
        pi = philox.givens_permutation(n, seed, 0)
        assert sorted(pi.tolist()) == list(range(n))
        counts[np.arange(n), pi] += 1
    # chi-square over the n x n position table ((n-1)^2 = 25 degrees of freedom; 60 is p < 1e-4)
    expect = trials / n
    chi2 = np.sum((counts - expect) ** 2 / expect)
    assert chi2 < 60, chi2
    th = philox.givens_angles(20001, 12, 1)
    assert th.min() >= 0.0 and th.max() < 2 * np.pi
    assert abs(np.mean(np.cos(th))) < 0.03 and abs(np.mean(np.sin(th))) < 0.03


def test_range_captured_at_exact_rank():
    m, n, r, l = 60, 64, 7, 12
    rng = np.random.default_rng(13)
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    Q = gsrft.gsrft_range_finder(A, l, 14)
    assert np.linalg.norm(A - Q @ (Q.T @ A), 2) <= 1e-12 * np.linalg.norm(A, 2)
    assert np.linalg.norm(Q.T @ Q - np.eye(l), 2) <= 1e-12
