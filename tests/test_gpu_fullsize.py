"""The two large workloads at full size, in the launch configuration the benchmark times, against
the FP64 oracle run on exactly the matrix the GPU read (marked gpu):

  * power iteration: FP32 16384 x 8192, sigma_j = 1/j, k = 100, p = 20, q = 2, the four hot-path
    calls with their split of K, in FP32 and in bf16x3 arithmetic;
  * SRFT workload: FP32 32768 x 16384, sigma_1..50 in [1, 2], a flat 1e-3 tail, k = 50, p = 78,
    q = 0, with the SRFT and with the Gaussian sketch.

The oracle finishes these sizes in seconds to a minute on the host.  The spectral norm of each
residual A - U_k S_k V_k^T is measured by the benchmark's evaluator (FP64 block subspace iteration
on the GPU, checked against the exact norm in test_evaluator.py), the same evaluator for the GPU's
and the oracle's factors.

Tolerances.  FP32 path: every retained singular value within 1e-5 relative of the oracle's (the
stated budget, no absolute floor: at these spectra sigma_k is far above FP32 resolution), the
residual within 1% of the oracle's, in both directions.  bf16x3 path, also against the oracle: the
split a = hi + lo leaves each product with a relative error up to 2^-16 (the dropped lo * lo term
and the roundings of hi and lo), so B = Q* A carries an absolute error of about
2^-16 sqrt(m) ||Q col|| ||A col|| <= 2^-16 ||A||_2 per entry direction, and by Weyl's inequality each
singular value moves by at most about 2^-16 sigma_1; relative to sigma_k = 1/100 that is
1.5e-3.  Asserted: |dsigma_j| <= 2^-16 sigma_1 + 1e-5 sigma_j, and the residual within 1% of the
oracle's (the metric's "equal ||A - U S V*|| / sigma_(k+1)").  Measured errors are printed.
"""

import numpy as np
import pytest
import torch

import bench
import paper_0909_4061_amd as rs
from oracle import evaluate, philox, rsvd as orsvd
from workloads import CONFIGS, build_matrix_torch, spectrum

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
M, N, K, P, Q, SEED = 16384, 8192, 100, 20, 2, 3


def _res(A, U, S, V):
    return bench.spectral_norm_residual(A, U.to(A.device), S.to(A.device), V.to(A.device))


@pytest.fixture(scope="module")
def full():
    sigma = spectrum("inv", N)
    A = build_matrix_torch(M, N, sigma, seed=SEED, dtype=torch.float32, device=DEV)
    out = {prec: rs.rsvd(A, K, P, Q, prec=prec, seed=SEED) for prec in ("native", "bf16x3")}
    torch.cuda.synchronize()
    assert rs.device_status(DEV) & ~rs.RSVD_FLAG_SHIFTED == 0
    ref = orsvd.rsvd(A.double().cpu().numpy(), K, P, Q, seed=SEED, stream=0, dtype=np.float32)
    res = {prec: _res(A, *o) for prec, o in out.items()}
    res["oracle"] = _res(A, *(torch.from_numpy(ref[x]) for x in ("Uk", "Sk", "Vk")))
    return dict(sigma=sigma, out=out, ref=ref, res=res)


def test_fp32_full_size_matches_oracle(full):
    S = full["out"]["native"][1].double().cpu().numpy()
    Sr = full["ref"]["Sk"]
    rel = np.abs(S - Sr) / Sr
    r, r_ref = full["res"]["native"], full["res"]["oracle"]
    print(f"FP32 16384x8192 q=2: max sigma rel err vs oracle {rel.max():.3e}, "
          f"residual {r:.6e} vs oracle {r_ref:.6e} (ratio {r / r_ref:.6f})")
    assert np.all(rel <= 1e-5), rel.max()
    assert abs(r - r_ref) <= 0.01 * r_ref, (r, r_ref)
    assert r >= 0.99 * full["sigma"][K]  # Mirsky (to the evaluator's accuracy): nothing beats sigma_(k+1)
    U = full["out"]["native"][0].double().cpu().numpy()
    assert evaluate.orthonormality_error(U) <= 1e-5


def test_bf16x3_full_size_matches_oracle(full):
    Sb = full["out"]["bf16x3"][1].double().cpu().numpy()
    Sr = full["ref"]["Sk"]
    err = np.abs(Sb - Sr)
    r, r_ref = full["res"]["bf16x3"], full["res"]["oracle"]
    print(f"bf16x3 16384x8192 q=2: max sigma rel err vs oracle {np.max(err / Sr):.3e}, max abs "
          f"{err.max():.3e} (sigma_1 {Sr[0]:.3e}), residual ratio vs oracle {r / r_ref:.6f}")
    assert np.all(err <= 2.0 ** -16 * Sr[0] + 1e-5 * Sr), np.max(err / (2.0 ** -16 * Sr[0] + 1e-5 * Sr))
    assert abs(r - r_ref) <= 0.01 * r_ref, (r, r_ref)
    Ub = full["out"]["bf16x3"][0].double().cpu().numpy()
    assert evaluate.orthonormality_error(Ub) <= 1e-5


@pytest.fixture(scope="module")
def srft_full():
    cfg = CONFIGS["srft_32768x16384"]
    sig = spectrum(cfg.spectrum, min(cfg.m, cfg.n))
    A = build_matrix_torch(cfg.m, cfg.n, sig, dtype=torch.float32, device=DEV)
    seed = 0x09094061
    out = {sk: rs.rsvd(A, cfg.k, cfg.p, 0, sketch=sk, seed=seed, prec="native") for sk in ("srft", "gaussian")}
    torch.cuda.synchronize()
    assert rs.device_status(DEV) & ~rs.RSVD_FLAG_SHIFTED == 0
    A64 = A.double().cpu().numpy()
    refs = {sk: orsvd.rsvd(A64, cfg.k, cfg.p, 0, seed=seed, stream=0, dtype=np.float32, sketch=sk)
            for sk in ("srft", "gaussian")}
    del A64
    res = {sk: _res(A, *o) for sk, o in out.items()}
    res_ref = {sk: _res(A, *(torch.from_numpy(refs[sk][x]) for x in ("Uk", "Sk", "Vk"))) for sk in refs}
    return dict(cfg=cfg, out=out, refs=refs, res=res, res_ref=res_ref)


@pytest.mark.parametrize("sketch", ["srft", "gaussian"])
def test_srft_workload_full_size_matches_oracle(srft_full, sketch):
    cfg = srft_full["cfg"]
    S = srft_full["out"][sketch][1].double().cpu().numpy()
    Sr = srft_full["refs"][sketch]["Sk"]
    rel = np.abs(S - Sr) / Sr
    r, r_ref = srft_full["res"][sketch], srft_full["res_ref"][sketch]
    print(f"{sketch} 32768x16384 l=128: max sigma rel err vs oracle {rel.max():.3e}, "
          f"residual {r:.6e} vs oracle {r_ref:.6e} (ratio {r / r_ref:.6f})")
    assert np.all(rel <= 1e-5), rel.max()
    assert abs(r - r_ref) <= 0.01 * r_ref, (r, r_ref)
    U = srft_full["out"][sketch][0].double().cpu().numpy()
    assert evaluate.orthonormality_error(U) <= 1e-5
    assert S.shape == (cfg.k,)
