"""The benchmark's residual measurement (FP64 block subspace iteration with a final Rayleigh-Ritz
step, run by torch) against the oracle's exact spectral norm, on the CPU.  The measurement reports
||A - U S V*||_2 / sigma_(k+1), so an underestimate would flatter the GPU path: the evaluator must
agree with the dense-SVD norm to well below the 1% the residual parity checks resolve (asserted:
1e-6 relative).

Matrices are U diag(sigma) V^T with the decay profiles of the workloads (1/j, a gap, e^{-j/r}); the
factors are rank-k truncations of the exact SVD perturbed by FP32-level noise (the kind of factors
a GPU path returns), and a random rank-k factorization far from optimal."""

import numpy as np
import pytest
import torch

import bench
from oracle import evaluate
from workloads import build_matrix, spectrum


def _factors(A64, k, noise, rng):
    U, s, Vt = np.linalg.svd(A64, full_matrices=False)
    U, s, V = U[:, :k], s[:k], Vt[:k].T
    if noise:
        U = U + noise * rng.standard_normal(U.shape)
        V = V + noise * rng.standard_normal(V.shape)
        s = s * (1 + noise * rng.standard_normal(k))
    return U, s, V


@pytest.mark.parametrize("kind,m,n,k,noise", [("inv", 1200, 700, 50, 6e-8), ("inv", 900, 900, 100, 0.0),
                                              ("gap", 1000, 600, 50, 6e-8), ("exp", 800, 500, 20, 6e-8),
                                              ("inv", 1000, 500, 30, 1e-3)])
def test_spectral_norm_residual_matches_exact(kind, m, n, k, noise):
    rng = np.random.default_rng(m + n + k)
    if kind == "gap":
        sigma = np.r_[np.sort(rng.uniform(1, 2, 50))[::-1], np.abs(1e-3 * (1 + 0.1 * rng.standard_normal(n - 50)))]
    elif kind == "exp":
        sigma = spectrum("exp_r", n, rate=6.0)
    else:
        sigma = spectrum("inv", n)
    A64 = build_matrix(m, n, sigma, seed=m + k)
    U, s, V = _factors(A64, k, noise, rng)
    exact = evaluate.residual_usv(A64, U, s, V)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x))
    meas = bench.spectral_norm_residual(t(A64), t(U), t(s), t(V))
    assert abs(meas - exact) <= 1e-6 * exact, (meas, exact)


def test_spectral_norm_residual_random_factorization():
    # a residual whose top singular values are not separated from the next ones
    rng = np.random.default_rng(5)
    A64 = rng.standard_normal((600, 400))
    U, V = rng.standard_normal((600, 10)), rng.standard_normal((400, 10))
    s = rng.uniform(0.5, 1.0, 10)
    exact = evaluate.residual_usv(A64, U, s, V)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x))
    meas = bench.spectral_norm_residual(t(A64), t(U), t(s), t(V))
    assert meas <= exact * (1 + 1e-12)  # a Rayleigh-Ritz value never exceeds the norm
    assert meas >= 0.995 * exact, (meas, exact)
