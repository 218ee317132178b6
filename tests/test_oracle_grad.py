"""Pins of the reference gradient (oracle.rsvd_grad), on the CPU.

* its forward equals the numpy oracle's rSVD (singular values, and vectors
  after sign normalization);
* central finite differences of the loss along random directions agree with
  the autograd gradient (64 x 32 instances, FP64);
* closed form: with l = n and q = 0, range(Q) = range(A), so the loss
  sum_i w_i sigma_i equals that of the exact SVD and its gradient is
  U_k diag(w) V_k^T (the derivative of a simple singular value is u v^T).
"""

import numpy as np
import pytest

from oracle import philox, rsvd as orsvd
from oracle import rsvd_grad as og
from workloads import build_matrix, spectrum


def _instance(m, n, k, p, seed, kind="invsqrt"):
    A = build_matrix(m, n, spectrum(kind, min(m, n)), seed=seed)
    rng = np.random.default_rng(seed)
    T = rng.standard_normal((m, n))
    w = rng.uniform(0.0, 1.0, k)
    Om = philox.gaussian_omega(n, k + p, seed=seed)
    return A, T, w, Om


@pytest.mark.parametrize("q", [0, 1])
def test_forward_matches_numpy_oracle(q):
    import torch
    A, _, _, Om = _instance(80, 50, 6, 4, 3)
    U, S, V = og.rsvd_torch(torch.tensor(A), 6, 4, q, torch.tensor(Om))
    ref = orsvd.rsvd(A, 6, 4, q, Omega=Om)
    np.testing.assert_allclose(S.numpy(), ref["Sk"], rtol=1e-12)
    Ug, Vg = orsvd.normalize_signs(U.numpy(), V.numpy())
    Uo, Vo = orsvd.normalize_signs(ref["Uk"], ref["Vk"])
    np.testing.assert_allclose(Ug, Uo, atol=1e-10)
    np.testing.assert_allclose(Vg, Vo, atol=1e-10)


@pytest.mark.parametrize("q,seed", [(0, 1), (1, 2), (2, 5)])
def test_gradient_matches_finite_differences(q, seed):
    m, n, k, p = 64, 32, 8, 4
    A, T, w, Om = _instance(m, n, k, p, seed)
    _, G = og.loss_and_grad(A, k, p, q, Om, T, w)
    rng = np.random.default_rng(100 + seed)
    h = 1e-6
    for _ in range(3):
        E = rng.standard_normal((m, n))
        E /= np.linalg.norm(E)
        fd = (og.loss_value(A + h * E, k, p, q, Om, T, w) - og.loss_value(A - h * E, k, p, q, Om, T, w)) / (2 * h)
        an = float(np.sum(G * E))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_gradient_of_weighted_singular_values_closed_form():
    m, n, k = 40, 24, 5
    A = build_matrix(m, n, spectrum("exp_r", n, rate=6.0), seed=9)
    Om = philox.gaussian_omega(n, n, seed=9)      # l = n: the sketch spans range(A)
    w = np.random.default_rng(9).uniform(0.5, 1.5, k)
    T = np.zeros((m, n))
    # loss = ||U S V^T||^2 + sum w S = sum_i S_i^2 + w . S  ->  grad = U_k diag(2 S + w) V_k^T
    _, G = og.loss_and_grad(A, k, n - k, 0, Om, T, w)
    U, S, Vt = np.linalg.svd(A, full_matrices=False)
    expect = (U[:, :k] * (2 * S[:k] + w)[None, :]) @ Vt[:k]
    np.testing.assert_allclose(G, expect, atol=1e-10)
