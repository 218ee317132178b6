"""The single-pass eigendecomposition of a symmetric A on the GPU (rsvd_eigh_onepass: Algorithm 5.6
with the oversampled basis of the closing remark of Section 5.5), and the two-sided single pass for a
general A (rsvd_svd_onepass, Section 5.5), against the oracle
(oracle.single_pass) on the same A and the same test matrix Omega (the GPU draws Omega from
(seed, stream_id); the oracle draws the same values from its own generator), through the C ABI.

Tolerances.  The least-squares core B solves B (Q*Omega) = Q*Y; a perturbation dN of Q*Y (from the
rounding of Y = A Omega and of the products with Q) moves B by at most ||dN|| / sigma_min(Q*Omega)
(the bound behind the remark), and every eigenvalue by at most that (Weyl).  ||dN|| is bounded by
delta ||A|| ||Omega|| with delta = 2^-24 sqrt(n) (FP32 products), 2^-16 + 2^-24 sqrt(n) (bf16x3),
4 u_64 sqrt(n) (FP64), plus the same relative error again for the basis Q (it comes from Y);
the tests allow eps_B = 2 delta ||A|| ||Omega|| / sigma_min(Q*Omega) on eigenvalues and
2 eps_B / gap + 1e-5 (Davis-Kahan, plus the lift's rounding) on the sine of each eigenvector's
angle to the oracle's."""

import numpy as np
import pytest
import torch

import paper_0909_4061_amd as rs
from oracle import rsvd as orsvd, single_pass
from tests.gpu_common import to_np
from workloads import build_symmetric

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _case(n, lam, k, p, npd, seed, prec="native"):
    A = build_symmetric(n, lam, seed=seed, dtype=npd)
    A64 = A.astype(np.float64)
    At = torch.from_numpy(A).to(DEV)
    print(f"onepass n={n} k={k} p={p} {A.dtype} {prec}", flush=True)
    rs.device_status(DEV)
    U, L = rs.rsvd_eigh_onepass(At, k, p, prec=prec, seed=seed + 1)
    flags = rs.device_status(DEV)
    Om = orsvd.gaussian_test_matrix(n, k + p, seed + 1, 0, npd)
    Ur, Lr = single_pass.one_pass_eig(A64, Om, k)
    Q = single_pass.one_pass_basis(A64 @ Om, k)
    tau = np.linalg.svd(Q.T @ Om, compute_uv=False)[-1]
    B = single_pass.least_squares_core(Q, Om, A64 @ Om)
    return (to_np(U).astype(np.float64), to_np(L).astype(np.float64), flags, Ur, Lr, tau,
            np.linalg.norm(Om, 2), np.linalg.eigvalsh(B))


def _sin(u, r):
    u = u / np.linalg.norm(u)
    r = r / np.linalg.norm(r)
    return np.linalg.norm(u - np.dot(u, r) * r)


def _gaps(lam_all, picked):
    return np.array([np.min(np.abs(np.delete(lam_all, np.argmin(np.abs(lam_all - v))) - v)) for v in picked])


def _check(U, L, Ur, Lr, eps_b, B_eigs, orth_tol):
    err = np.max(np.abs(L - Lr))
    assert err <= eps_b, (err, eps_b)
    for j, g in enumerate(_gaps(B_eigs, Lr)):
        assert _sin(U[:, j], Ur[:, j]) <= 2 * eps_b / g + 1e-5, (j, _sin(U[:, j], Ur[:, j]), g)
    assert np.linalg.norm(U.T @ U - np.eye(U.shape[1]), 2) <= orth_tol
    return err


@pytest.mark.parametrize("p", [0, 8])
def test_onepass_fp64_matches_oracle(p):
    n, k = 300, 10
    j = np.arange(1, n + 1, dtype=np.float64)
    lam = (-1.0) ** j / j
    U, L, flags, Ur, Lr, tau, nom, Beig = _case(n, lam, k, p, np.float64, 91)
    eps_b = 2 * 4 * 2.0 ** -53 * np.sqrt(n) * 1.0 * nom / tau
    err = _check(U, L, Ur, Lr, eps_b, Beig, 1e-12)
    print(f"fp64 p={p}: sigma_min(Q*Omega) {tau:.3f}, max |lambda - ref| {err:.3e} (tol {eps_b:.3e})")
    assert flags == 0


@pytest.mark.parametrize("prec", ["native", "bf16x3"])
def test_onepass_fp32_matches_oracle(prec):
    n, k, p = 1000, 16, 10
    j = np.arange(1, n + 1, dtype=np.float64)
    lam = (-1.0) ** j / j
    U, L, flags, Ur, Lr, tau, nom, Beig = _case(n, lam, k, p, np.float32, 92, prec)
    delta = 2.0 ** -24 * np.sqrt(n) + (2.0 ** -16 if prec == "bf16x3" else 0.0)
    eps_b = 2 * delta * 1.0 * nom / tau
    err = _check(U, L, Ur, Lr, eps_b, Beig, 1e-5)
    print(f"fp32 {prec}: sigma_min(Q*Omega) {tau:.3f}, max |lambda - ref| {err:.3e} (tol {eps_b:.3e})")
    assert flags == 0


def test_onepass_exact_rank_fp64():
    n = 200
    lam = [2.0, -4.0, 1.0, -0.5, 3.0, 0.25]
    k, p = len(lam), 6
    U, L, flags, Ur, Lr, tau, nom, Beig = _case(n, lam, k, p, np.float64, 93)
    A64 = build_symmetric(n, lam, seed=93)
    expect = sorted(lam, key=lambda x: (-abs(x), -x))
    assert np.max(np.abs(L - expect)) <= 1e-11 * 4.0
    assert np.linalg.norm(A64 - (U * L[None, :]) @ U.T, 2) <= 1e-10 * 4.0
    # Y = A Omega has rank k < l: the orthonormalization inside the small SVD of Y shifts
    assert flags & ~rs.RSVD_FLAG_SHIFTED == 0


def test_onepass_largest_basis_fp32():
    # l = 128, the largest the library takes
    n, k, p = 600, 100, 28
    j = np.arange(1, n + 1, dtype=np.float64)
    lam = j ** -1.5
    U, L, flags, Ur, Lr, tau, nom, Beig = _case(n, lam, k, p, np.float32, 94)
    eps_b = 2 * 2.0 ** -24 * np.sqrt(n) * nom / tau
    err = np.max(np.abs(L - Lr))
    print(f"fp32 l=128: sigma_min {tau:.3f}, max |lambda - ref| {err:.3e} (tol {eps_b:.3e})")
    assert err <= eps_b
    assert np.linalg.norm(U.T @ U - np.eye(k), 2) <= 1e-4
    assert flags & ~rs.RSVD_FLAG_SHIFTED == 0


# --- the two-sided single pass for a general A (rsvd_svd_onepass) --------------------------------
# Omegat is drawn from the stream id with its top bit flipped.  The least-squares B moves by at most
# ||(dN1, dN2)|| / sqrt(sigma_min(M1)^2 + sigma_min(M2)^2) for perturbations dN of the right-hand
# sides (the bound pinned on the oracle), and every singular value by at most that (Weyl);
# ||dN|| <= delta ||A|| max(||Omega||, ||Omegat||) with delta as above.

def _two_sided_case(m, n, sigma, k, p, npd, seed, prec="native"):
    from workloads import build_matrix
    A = build_matrix(m, n, sigma, seed=seed, dtype=npd)
    A64 = A.astype(np.float64)
    l = k + p
    print(f"svd onepass {m}x{n} k={k} p={p} {A.dtype} {prec}", flush=True)
    rs.device_status(DEV)
    U, S, V = rs.rsvd_svd_onepass(torch.from_numpy(A).to(DEV), k, p, prec=prec, seed=seed + 1)
    flags = rs.device_status(DEV)
    Om = orsvd.gaussian_test_matrix(n, l, seed + 1, 0, npd)
    Omt = orsvd.gaussian_test_matrix(m, l, seed + 1, 1 << 63, npd)
    # the stacked least-squares system has 2 l^2 x l^2 entries: its normal-equation route beyond l = 64
    Ur, Sr, Vr = single_pass.two_sided_svd(A64, Om, Omt, k, solver="lstsq" if l <= 64 else "normal")
    Q, _ = orsvd.qr_pos(A64 @ Om)
    Qt, _ = orsvd.qr_pos(A64.T @ Omt)
    s1 = np.linalg.svd(Qt.T @ Om, compute_uv=False)[-1]
    s2 = np.linalg.svd(Q.T @ Omt, compute_uv=False)[-1]
    amp = max(np.linalg.norm(Om, 2), np.linalg.norm(Omt, 2)) / np.sqrt(s1 ** 2 + s2 ** 2)
    return A64, [to_np(t).astype(np.float64) for t in (U, S, V)], flags, (Ur, Sr, Vr), amp


@pytest.mark.parametrize("npd,prec", [(np.float64, "native"), (np.float32, "native"), (np.float32, "bf16x3")])
def test_svd_onepass_matches_oracle(npd, prec):
    m, n, k, p = (300, 200, 10, 8) if npd == np.float64 else (1200, 800, 16, 8)
    sigma = 1.0 / np.arange(1, min(m, n) + 1, dtype=np.float64)
    A64, (U, S, V), flags, (Ur, Sr, Vr), amp = _two_sided_case(m, n, sigma, k, p, npd, 95, prec)
    if npd == np.float64:
        delta = 4 * 2.0 ** -53 * np.sqrt(max(m, n))
    else:
        delta = 2.0 ** -24 * np.sqrt(max(m, n)) + (2.0 ** -16 if prec == "bf16x3" else 0.0)
    eps_b = 2 * delta * sigma[0] * amp
    err = np.max(np.abs(S - Sr))
    print(f"svd onepass {npd.__name__} {prec}: amplification {amp:.2f}, max |s - ref| {err:.3e} (tol {eps_b:.3e})")
    assert flags & ~rs.RSVD_FLAG_SHIFTED == 0
    assert err <= eps_b
    res = np.linalg.norm(A64 - (U * S[None, :]) @ V.T, 2)
    res_ref = np.linalg.norm(A64 - (Ur * Sr[None, :]) @ Vr.T, 2)
    assert abs(res - res_ref) <= 2 * eps_b + 1e-3 * res_ref, (res, res_ref)
    tol_o = 1e-12 if npd == np.float64 else 1e-5
    assert np.linalg.norm(U.T @ U - np.eye(k), 2) <= tol_o
    assert np.linalg.norm(V.T @ V - np.eye(k), 2) <= tol_o


def test_svd_onepass_exact_rank_fp64():
    m, n, r = 160, 120, 5
    sigma = np.zeros(n)
    sigma[:r] = np.linspace(3.0, 0.5, r)
    A64, (U, S, V), flags, _, _ = _two_sided_case(m, n, sigma, r, 3, np.float64, 96)
    assert np.max(np.abs(S - sigma[:r])) <= 1e-11 * 3.0
    assert np.linalg.norm(A64 - (U * S[None, :]) @ V.T, 2) <= 1e-10 * 3.0
    assert flags & ~rs.RSVD_FLAG_SHIFTED == 0


@pytest.mark.parametrize("m,n,k,p,npd", [
    (200, 300, 10, 8, np.float64),    # wide: the bases of the row space are the longer ones
    (160, 120, 12, 0, np.float64),    # p = 0: square relations (l x l coefficient matrices)
    (1000, 777, 24, 9, np.float32),   # ragged sizes, several tiles and a tail in every product
    (700, 500, 100, 28, np.float32),  # l = 128, the largest the library takes
])
def test_svd_onepass_shapes(m, n, k, p, npd):
    sigma = 1.0 / np.arange(1, min(m, n) + 1, dtype=np.float64) ** 1.5
    A64, (U, S, V), flags, (Ur, Sr, Vr), amp = _two_sided_case(m, n, sigma, k, p, npd, 97 + k)
    unit = 4 * 2.0 ** -53 if npd == np.float64 else 2.0 ** -24
    eps_b = 2 * unit * np.sqrt(max(m, n)) * sigma[0] * amp
    err = np.max(np.abs(S - Sr))
    print(f"svd onepass {m}x{n} k={k} p={p}: amplification {amp:.2f}, max |s - ref| {err:.3e} (tol {eps_b:.3e})")
    assert flags & ~rs.RSVD_FLAG_SHIFTED == 0
    assert err <= eps_b
    tol_o = 1e-12 if npd == np.float64 else 1e-4
    assert np.linalg.norm(U.T @ U - np.eye(k), 2) <= tol_o
    assert np.linalg.norm(V.T @ V - np.eye(k), 2) <= tol_o
    assert U.shape == (m, k) and V.shape == (n, k)
