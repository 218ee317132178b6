"""Stage B for symmetric and psd A on the GPU (rsvd_eigh: Algorithm 5.3, rsvd_nystrom: Algorithm 5.5)
against the oracle (oracle.herm) on the same A and the same basis Q, through the C ABI (marked gpu).

Q is made on the host by the oracle's range finder (Algorithm 4.1 in FP64) and rounded to the
element type; both sides read exactly those arrays.

Tolerances.  FP64: 1e-12 ||A|| on eigenvalues (u_64 sqrt(n) ||A|| is about 4e-15 ||A|| here).
FP32: the products A Q (one pass over A, relative error delta: 2^-24 sqrt(n) for FP32 products,
2^-16 for bf16x3 split products) and Q^T (A Q) (FP32, 2^-24 sqrt(n)) move B = Q^T A Q by at most
about (delta + 2^-24 sqrt(n)) ||A|| in norm, so by Weyl every eigenvalue of Algorithm 5.3 moves by
at most that much; the tests allow twice it.  Algorithm 5.5 also divides by the Cholesky factor of
B2, which amplifies the relative perturbation by up to kappa(B2): its eigenvalues are allowed
4 kappa(B2) (delta + 2^-24 sqrt(n)) ||A||.  Eigenvector columns with a gap g_j to the rest of the
spectrum are compared up to sign: sin-angle <= 2 eps_B / g_j + 1e-5 (Davis-Kahan with the same
perturbation eps_B, plus the rounding of the lift)."""

import numpy as np
import pytest
import torch

import paper_0909_4061_amd as rs
from oracle import herm, rsvd as orsvd
from tests.gpu_common import to_np
from workloads import build_symmetric

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _inputs(n, lam, l, npd, seed):
    A = build_symmetric(n, lam, seed=seed, dtype=npd)
    A64 = A.astype(np.float64)
    Om = orsvd.gaussian_test_matrix(n, l, seed + 1)
    Q = orsvd.randomized_range_finder(A64, Om).astype(npd)
    return A, A64, Q, Q.astype(np.float64)


def _run(fn, A, Q, k, prec="native"):
    At = torch.from_numpy(A).to(DEV)
    Qt = torch.from_numpy(np.ascontiguousarray(Q)).to(DEV)
    print(f"{fn.__name__} n={A.shape[0]} l={Q.shape[1]} k={k} {A.dtype} {prec}", flush=True)
    rs.device_status(DEV)  # clear
    U, Lam = fn(At, Qt, k, prec=prec)
    flags = rs.device_status(DEV)
    return to_np(U).astype(np.float64), to_np(Lam).astype(np.float64), flags


def _gaps(lam_all, picked):
    out = []
    for v in picked:
        d = np.abs(lam_all - v)
        d = d[d > 0]
        out.append(np.min(d) if d.size else np.inf)
    return np.array(out)


def _check_vectors(Ug, Ur, gaps, eps_b, extra=1e-5):
    # sin of the angle between column j of each, from the component of the GPU's (normalized)
    # vector orthogonal to the oracle's (stable where 1 - cos^2 is not)
    for j in range(Ug.shape[1]):
        u = Ug[:, j] / np.linalg.norm(Ug[:, j])
        r = Ur[:, j] / np.linalg.norm(Ur[:, j])
        sin = np.linalg.norm(u - np.dot(u, r) * r)
        assert sin <= 2 * eps_b / gaps[j] + extra, (j, sin, gaps[j])


def _orth(U):
    return np.linalg.norm(U.T @ U - np.eye(U.shape[1]), 2)


def test_eigh_fp64_matches_oracle():
    n, k, p = 300, 10, 6
    j = np.arange(1, n + 1, dtype=np.float64)
    lam = (-1.0) ** j / j
    A, A64, Q, Q64 = _inputs(n, lam, k + p, np.float64, 61)
    U, L, flags = _run(rs.rsvd_eigh, A, Q, k)
    Ur, Lr = herm.direct_eig(A64, Q64, k)
    nA = np.abs(lam).max()
    assert flags == 0
    assert np.max(np.abs(L - Lr)) <= 1e-12 * nA, (L, Lr)
    B = herm.hermitian_part(Q64.T @ A64 @ Q64)
    _check_vectors(U, Ur, _gaps(np.linalg.eigvalsh(B), Lr), 1e-12 * nA, extra=1e-10)
    assert _orth(U) <= 1e-12


@pytest.mark.parametrize("prec", ["native", "bf16x3"])
def test_eigh_fp32_matches_oracle(prec):
    n, k, p = 1000, 16, 8
    j = np.arange(1, n + 1, dtype=np.float64)
    lam = (-1.0) ** j / j
    A, A64, Q, Q64 = _inputs(n, lam, k + p, np.float32, 62)
    U, L, flags = _run(rs.rsvd_eigh, A, Q, k, prec)
    Ur, Lr = herm.direct_eig(A64, Q64, k)
    nA = np.abs(lam).max()
    delta = 2.0 ** -24 * np.sqrt(n) if prec == "native" else 2.0 ** -16
    eps_b = (delta + 2.0 ** -24 * np.sqrt(n)) * nA
    err = np.max(np.abs(L - Lr))
    print(f"eigh {prec}: max |lambda - ref| {err:.3e} (tol {2 * eps_b:.3e})")
    assert flags == 0
    assert err <= 2 * eps_b
    B = herm.hermitian_part(Q64.T @ A64 @ Q64)
    _check_vectors(U, Ur, _gaps(np.linalg.eigvalsh(B), Lr), eps_b)
    assert _orth(U) <= 1e-5


def test_eigh_exact_rank_and_order_fp64():
    # rank 5 < l: three kept eigenvalues at roundoff; the largest magnitude is negative
    n, k, p = 200, 8, 4
    lam = [3.0, -5.0, 1.0, -0.5, 2.0]
    A, A64, Q, Q64 = _inputs(n, lam, k + p, np.float64, 63)
    U, L, flags = _run(rs.rsvd_eigh, A, Q, k)
    assert flags & ~rs.RSVD_FLAG_SHIFTED == 0
    expect = sorted(lam, key=lambda x: (-abs(x), -x))
    assert np.max(np.abs(L[:5] - expect)) <= 1e-12 * 5.0
    assert np.max(np.abs(L[5:])) <= 1e-12 * 5.0
    assert _orth(U) <= 1e-12
    assert np.linalg.norm(A64 - (U * L[None, :]) @ U.T, 2) <= 1e-11 * 5.0


def test_nystrom_fp64_matches_oracle():
    n, k, p = 300, 10, 6
    j = np.arange(1, n + 1, dtype=np.float64)
    lam = 1.0 / j
    A, A64, Q, Q64 = _inputs(n, lam, k + p, np.float64, 64)
    U, L, flags = _run(rs.rsvd_nystrom, A, Q, k)
    Ur, Lr = herm.nystrom_eig(A64, Q64, k)
    assert flags == 0
    assert np.max(np.abs(L - Lr)) <= 1e-12, (L, Lr)
    F, _ = herm.nystrom_factor(A64, Q64)
    lam_f = np.linalg.svd(F, compute_uv=False) ** 2
    _check_vectors(U, Ur, _gaps(lam_f, Lr), 1e-12, extra=1e-10)
    assert _orth(U) <= 1e-12


@pytest.mark.parametrize("prec", ["native", "bf16x3"])
def test_nystrom_fp32_matches_oracle(prec):
    n, k, p = 1000, 16, 8
    j = np.arange(1, n + 1, dtype=np.float64)
    lam = 1.0 / j
    A, A64, Q, Q64 = _inputs(n, lam, k + p, np.float32, 65)
    U, L, flags = _run(rs.rsvd_nystrom, A, Q, k, prec)
    Ur, Lr = herm.nystrom_eig(A64, Q64, k)
    B2 = herm.hermitian_part(Q64.T @ A64 @ Q64)
    ev = np.linalg.eigvalsh(B2)
    kappa = ev[-1] / ev[0]
    delta = 2.0 ** -24 * np.sqrt(n) if prec == "native" else 2.0 ** -16
    eps_b = kappa * (delta + 2.0 ** -24 * np.sqrt(n)) * lam[0]
    err = np.max(np.abs(L - Lr))
    print(f"nystrom {prec}: kappa(B2) {kappa:.1f}, max |lambda - ref| {err:.3e} (tol {4 * eps_b:.3e})")
    assert flags == 0
    assert err <= 4 * eps_b
    F, _ = herm.nystrom_factor(A64, Q64)
    lam_f = np.linalg.svd(F, compute_uv=False) ** 2
    _check_vectors(U, Ur, _gaps(lam_f, Lr), 2 * eps_b)
    assert _orth(U) <= 1e-5


def test_nystrom_singular_core_is_shifted():
    # rank 4 < l: B2 = Q^T A Q is singular; the Cholesky factorization restarts on B2 + s I
    n, k, p = 160, 4, 6
    lam = [4.0, 2.0, 1.0, 0.5]
    A, A64, Q, Q64 = _inputs(n, lam, k + p, np.float64, 66)
    U, L, flags = _run(rs.rsvd_nystrom, A, Q, k)
    assert np.all(np.isfinite(U)) and np.all(np.isfinite(L))
    if flags & rs.RSVD_FLAG_SHIFTED:
        assert flags & ~rs.RSVD_FLAG_SHIFTED == 0
    # the shift is at the level of 1e-11 of the trace: the nonzero eigenvalues survive
    assert np.max(np.abs(L - np.array(lam))) <= 1e-6 * 4.0, L
    assert _orth(U) <= 1e-8


@pytest.mark.parametrize("fn", ["eigh", "nystrom"])
def test_small_basis_k_equals_l_fp32(fn):
    n, k = 257, 4
    j = np.arange(1, n + 1, dtype=np.float64)
    lam = 1.0 / j ** 2 if fn == "nystrom" else (-1.0) ** j / j ** 2
    A, A64, Q, Q64 = _inputs(n, lam, k, np.float32, 67)
    f = rs.rsvd_eigh if fn == "eigh" else rs.rsvd_nystrom
    U, L, flags = _run(f, A, Q, k)
    Ur, Lr = (herm.direct_eig if fn == "eigh" else herm.nystrom_eig)(A64, Q64, k)
    assert flags == 0
    assert np.max(np.abs(L - Lr)) <= 1e-4 * np.abs(lam).max(), (L, Lr)
    assert _orth(U) <= 1e-5
