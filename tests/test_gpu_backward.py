"""Hand-written adjoint of the fixed-Omega rSVD (rsvd_backward, through
RSVDFunction) vs the FP64 reference gradient of oracle.rsvd_grad (marked gpu).

Loss (the differentiable workload): L = ||U_k diag(S_k) V_k^T - T||_F^2 +
sum_i w_i S_i, T standard Gaussian, w uniform in [0, 1]; its gradient in A
does not depend on sign conventions.  Comparisons use the relative Frobenius
error of dL/dA.  Tolerance 64 l u for FP64 and FP32 products (u the unit
roundoff of the element type) and 2 l 2^-16 for bf16x3 products (2^-16 is the
worst-case relative error of the split x = hi + lo, hi and lo rounded to BF16):
the adjoint is a fixed sequence of products in the element type plus l x l
algebra in FP64, and on the well-separated spectra used here (sigma_j =
j^-1/2) its error stays of the order of the forward's, l u.  Measured: about
1e-14 in FP64; 0.5 to 3 l 2^-24 in FP32; 0.01 to 0.33 l 2^-16 with bf16x3
products (the largest for the 96 x 80, q = 2 case), so the bf16x3 bound keeps a
margin of six over the worst case seen.
Near-degenerate sigma_k, sigma_(k+1) would multiply it by up to
sigma_1^2 / (sigma_k^2 - sigma_(k+1)^2) (the F matrix of the SVD derivative)
and are not used.
"""

import numpy as np
import pytest
import torch

import paper_0909_4061_amd as rs
from oracle import philox, rsvd as orsvd
from oracle import rsvd_grad as og
from tests.gpu_common import to_np
from workloads import build_matrix, build_matrix_torch, spectrum

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
UNIT = {torch.float64: 2.0 ** -53, torch.float32: 2.0 ** -24}


def _gpu_grad(A, k, p, q, seed, T, w, prec="native"):
    At = A.detach().clone().requires_grad_(True)
    U, S, V = rs.rsvd(At, k, p, q, seed=seed, prec=prec)
    L = ((U * S[None, :]) @ V.T - T).square().sum() + (w * S).sum()
    L.backward()
    torch.cuda.synchronize()
    return At.grad


def _tol(sigma, k, l, dtype, prec="native"):
    del sigma, k
    # bf16x3 products: x = hi + lo carries a relative error up to 2^-16 per element
    return 2.0 * l * 2.0 ** -16 if prec == "bf16x3" else 64.0 * l * UNIT[dtype]


def _case(m, n, k, p, q, dtype, kind, seed, prec="native"):
    sig = spectrum(kind, min(m, n))
    A64 = build_matrix(m, n, sig, seed=seed, dtype=np.float32 if dtype == torch.float32 else np.float64)
    rng = np.random.default_rng(seed)
    T = rng.standard_normal((m, n))
    w = rng.uniform(0.0, 1.0, k)
    A = torch.from_numpy(A64).to(DEV)
    G = _gpu_grad(A, k, p, q, seed, torch.from_numpy(T).to(DEV, dtype), torch.from_numpy(w).to(DEV, dtype), prec)
    Om = philox.round_to_dtype(philox.gaussian_omega(n, k + p, seed=seed),
                               np.float32 if dtype == torch.float32 else np.float64)
    _, Gref = og.loss_and_grad(to_np(A).astype(np.float64), k, p, q, Om, T, w)
    err = np.linalg.norm(to_np(G).astype(np.float64) - Gref) / np.linalg.norm(Gref)
    return err, _tol(sig, k, k + p, dtype, prec)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_backward_fp64_matches_reference(q):
    err, tol = _case(300, 200, 10, 6, q, torch.float64, "invsqrt", seed=20 + q)
    assert err <= tol, (err, tol)
    assert rs.device_status(DEV) == 0


# (96, 80, 16, 8, 2): gA's contraction (2q + 2) l = 144 exceeds max(m, n) and m is
# less than one 128-row block
@pytest.mark.parametrize("m,n,k,p,q", [(512, 256, 16, 8, 1), (333, 130, 20, 12, 0), (257, 257, 30, 10, 2),
                                       (96, 80, 16, 8, 2)])
@pytest.mark.parametrize("prec", ["native", "bf16x3"])
def test_backward_fp32_matches_reference(m, n, k, p, q, prec):
    err, tol = _case(m, n, k, p, q, torch.float32, "invsqrt", seed=m + n, prec=prec)
    print(f"backward fp32 {prec} {m}x{n} k={k} p={p} q={q}: rel err {err:.3e} (tol {tol:.3e}, "
          f"{err / (k + p) / 2.0 ** -16:.3f} l 2^-16)")
    assert err <= tol, (err, tol)
    assert rs.device_status(DEV) == 0


def test_backward_full_size_differentiable_workload():
    # one 4096 x 2048 FP32 matrix of the differentiable workload: sigma_j = j^-1/2, k = 64, p = 16, q = 1
    m, n, k, p, q = 4096, 2048, 64, 16, 1
    sig = spectrum("invsqrt", n)
    A = build_matrix_torch(m, n, sig, seed=77, dtype=torch.float32, device=DEV)
    rng = np.random.default_rng(77)
    T = rng.standard_normal((m, n))
    w = rng.uniform(0.0, 1.0, k)
    G = _gpu_grad(A, k, p, q, 5, torch.from_numpy(T).to(DEV, torch.float32),
                  torch.from_numpy(w).to(DEV, torch.float32))
    Om = philox.round_to_dtype(philox.gaussian_omega(n, k + p, seed=5), np.float32)
    _, Gref = og.loss_and_grad(to_np(A).astype(np.float64), k, p, q, Om, T, w)
    err = np.linalg.norm(to_np(G).astype(np.float64) - Gref) / np.linalg.norm(Gref)
    assert err <= _tol(sig, k, k + p, torch.float32), err


def test_backward_closed_form_full_sample():
    # l = n and q = 0: range(Q) = range(A), and L = sum S_i^2 + w . S has
    # gradient U_k diag(2 S + w) V_k^T
    m, n, k = 120, 48, 6
    A64 = build_matrix(m, n, spectrum("exp_r", n, rate=8.0), seed=31)
    A = torch.from_numpy(A64).to(DEV)
    w = np.random.default_rng(31).uniform(0.5, 1.5, k)
    G = _gpu_grad(A, k, n - k, 0, 3, torch.zeros(m, n, dtype=torch.float64, device=DEV),
                  torch.from_numpy(w).to(DEV))
    U, S, Vt = np.linalg.svd(A64, full_matrices=False)
    expect = (U[:, :k] * (2 * S[:k] + w)[None, :]) @ Vt[:k]
    np.testing.assert_allclose(to_np(G), expect, atol=1e-10)


def test_backward_matches_finite_differences_of_gpu_forward():
    m, n, k, p, q = 64, 32, 8, 4, 1
    A64 = build_matrix(m, n, spectrum("invsqrt", n), seed=12)
    rng = np.random.default_rng(12)
    T = torch.from_numpy(rng.standard_normal((m, n))).to(DEV)
    w = torch.from_numpy(rng.uniform(0, 1, k)).to(DEV)
    A = torch.from_numpy(A64).to(DEV)
    G = to_np(_gpu_grad(A, k, p, q, 9, T, w))

    def loss(X):
        U, S, V = rs.rsvd(X, k, p, q, seed=9)
        return float(((U * S[None, :]) @ V.T - T).square().sum() + (w * S).sum())

    h = 1e-6
    for _ in range(3):
        E = torch.from_numpy(rng.standard_normal((m, n))).to(DEV)
        E /= torch.linalg.norm(E)
        fd = (loss(A + h * E) - loss(A - h * E)) / (2 * h)
        an = float(np.sum(G * to_np(E)))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


@pytest.mark.parametrize("dtype,prec", [(torch.float64, "native"), (torch.float32, "bf16x3")])
def test_kept_forward_state_matches_recomputation(dtype, prec):
    # rsvd_backward_kept, which skips the recomputation, returns rsvd_backward's gA bit
    # for bit, also when called twice.  rsvd_forward_kept orthonormalizes every basis of
    # the power scheme by CholeskyQR2 (the adjoint differentiates exact QR factors), where
    # the hot path takes one pass for the bases inside it: the same factorization up to
    # the element type's rounding.
    m, n, k, p, q = 700, 300, 12, 8, 2
    A64 = build_matrix(m, n, spectrum("invsqrt", n), seed=14,
                       dtype=np.float32 if dtype == torch.float32 else np.float64)
    A = torch.from_numpy(A64).to(DEV)
    rng = np.random.default_rng(14)
    gU = torch.from_numpy(rng.standard_normal((m, k))).to(DEV, dtype)
    gS = torch.from_numpy(rng.standard_normal(k)).to(DEV, dtype)
    gV = torch.from_numpy(rng.standard_normal((n, k))).to(DEV, dtype)
    U0, S0, V0 = rs.rsvd(A, k, p, q, seed=6, prec=prec)
    U, S, V, ws = rs.rsvd_forward_kept(A, k, p, q, seed=6, prec=prec)
    g_re = rs.rsvd_backward(A, gU, gS, gV, k, p, q, seed=6, prec=prec)
    g1 = rs.rsvd_backward_kept(A, gU, gS, gV, k, p, q, ws, seed=6, prec=prec)
    g2 = rs.rsvd_backward_kept(A, gU, gS, gV, k, p, q, ws, seed=6, prec=prec)
    torch.cuda.synchronize()
    for a, b in ((g1, g_re), (g2, g_re)):
        assert torch.equal(a, b)
    fp64 = dtype == torch.float64
    S, S0 = to_np(S).astype(np.float64), to_np(S0).astype(np.float64)
    assert np.max(np.abs(S - S0) / S0) <= (1e-12 if fp64 else 1e-5)
    Uk, Vk = orsvd.normalize_signs(to_np(U).astype(np.float64), to_np(V).astype(np.float64))
    U0, V0 = orsvd.normalize_signs(to_np(U0).astype(np.float64), to_np(V0).astype(np.float64))
    assert max(np.max(np.abs(Uk - U0)), np.max(np.abs(Vk - V0))) <= (1e-9 if fp64 else 1e-3)
