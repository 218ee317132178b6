"""The power-iteration workload at its full size, in the launch configuration
the benchmark times (FP32 16384 x 8192, sigma_j = 1/j, k = 100, p = 20, q = 2,
the four hot-path calls with their split of K), against the FP64 oracle run
on exactly the matrix the GPU read (marked gpu).

The oracle finishes this size in seconds on the host.  The spectral norm of
each residual A - U_k S_k V_k^T is measured on the GPU in FP64 by block power
iteration on the implicit operator (a measurement, the same evaluator for the
GPU's and the oracle's factors).  Tolerances as for the batched parity tests:
FP32 singular values within 1e-5 sigma_j + (4 sqrt(m) + 2 l) u sigma_1, the
residual within 1% of the oracle's; the bf16x3 path within 1% of the FP32
path's residual and 1e-3 of its singular values.
"""

import numpy as np
import pytest
import torch

import paper_0909_4061_amd as rs
from oracle import evaluate, rsvd as orsvd
from workloads import build_matrix_torch, spectrum

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
M, N, K, P, Q, SEED = 16384, 8192, 100, 20, 2, 3


def _residual_2norm(A64, U, S, V, iters=40, block=8):
    """||A - U diag(S) V^T||_2, FP64 block power iteration on the GPU."""
    U, S, V = (t.to(DEV, torch.float64) for t in (U, S, V))
    gen = torch.Generator(device=DEV)
    gen.manual_seed(11)
    X = torch.randn(A64.shape[1], block, generator=gen, device=DEV, dtype=torch.float64)
    for _ in range(iters):
        X, _ = torch.linalg.qr(X)
        Y = A64 @ X - U @ (S[:, None] * (V.T @ X))
        X = A64.T @ Y - V @ (S[:, None] * (U.T @ Y))
    X, _ = torch.linalg.qr(X)
    Y = A64 @ X - U @ (S[:, None] * (V.T @ X))
    return float(torch.linalg.svdvals(Y)[0])


@pytest.fixture(scope="module")
def full():
    sigma = spectrum("inv", N)
    A = build_matrix_torch(M, N, sigma, seed=SEED, dtype=torch.float32, device=DEV)
    out = {prec: rs.rsvd(A, K, P, Q, prec=prec, seed=SEED) for prec in ("native", "bf16x3")}
    torch.cuda.synchronize()
    assert rs.device_status(DEV) & ~rs.RSVD_FLAG_SHIFTED == 0
    A64 = A.double()
    ref = orsvd.rsvd(A64.cpu().numpy(), K, P, Q, seed=SEED, stream=0, dtype=np.float32)
    res = {prec: _residual_2norm(A64, *o) for prec, o in out.items()}
    res["oracle"] = _residual_2norm(A64, *(torch.from_numpy(ref[x]) for x in ("Uk", "Sk", "Vk")))
    return dict(sigma=sigma, out=out, ref=ref, res=res)


def test_fp32_full_size_matches_oracle(full):
    S = full["out"]["native"][1].double().cpu().numpy()
    Sr = full["ref"]["Sk"]
    floor = (4.0 * np.sqrt(M) + 2.0 * (K + P)) * 2.0 ** -24 * Sr[0]
    assert np.all(np.abs(S - Sr) <= 1e-5 * Sr + floor), np.max(np.abs(S - Sr) / (1e-5 * Sr + floor))
    r, r_ref = full["res"]["native"], full["res"]["oracle"]
    assert abs(r - r_ref) <= 0.01 * r_ref + floor, (r, r_ref)
    assert r >= 0.99 * full["sigma"][K]  # Mirsky (to the evaluator's accuracy): nothing beats sigma_(k+1)
    U = full["out"]["native"][0].double().cpu().numpy()
    assert evaluate.orthonormality_error(U) <= 1e-5


def test_bf16x3_full_size_matches_fp32_path(full):
    Sb = full["out"]["bf16x3"][1].double().cpu().numpy()
    S32 = full["out"]["native"][1].double().cpu().numpy()
    assert np.max(np.abs(Sb - S32) / S32) < 1e-3
    assert abs(full["res"]["bf16x3"] - full["res"]["native"]) <= 0.01 * full["res"]["native"]
    Ub = full["out"]["bf16x3"][0].double().cpu().numpy()
    assert evaluate.orthonormality_error(Ub) <= 1e-5
