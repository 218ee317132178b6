"""The fixed-precision range finder (rsvd_range_finder_tol: Algorithm 4.2 in doubling blocks) against
its oracle (oracle.adaptive.blocked_adaptive_range_finder) on the same matrix and the same test
vectors, through the C ABI (marked gpu).

The two take the same decisions when every tested estimate is far from eps (the workloads below are
chosen so), hence the same basis size l; then the basis spans the same range and the estimate agrees.

FP64: estimate and residual ||(I - Q Q*) A|| within 1e-9 relative, Q orthonormal to 1e-13.

FP32 data.  The accepted estimate is 10 sqrt(2/pi) times the largest projected sample
||(I - Q Q*) A w||, here about 3e-5 of ||A w||: the projected samples are small differences of FP32
vectors and carry the products' rounding.  Error model: delta = 2^-24 sqrt(n) for FP32 products
(n-term accumulations, rounding errors of random sign), delta = 2^-16 for bf16x3 (the split
products' relative error).  A projected sample moves by at most about delta ||A w|| (triangle
inequality), the residual norm by at most about delta sigma_1 (Weyl), so the tests assert
    |est - est_oracle| <= 0.01 est_oracle + 10 sqrt(2/pi) delta max_i ||A w_i||,
    |res - res_oracle| <= 0.01 res_oracle + delta sigma_1,
the same l, res <= eps, and Q orthonormal to 1e-5.  (A plain FP32 re-computation of the same steps
on the host moves this estimate by 1.5%, the GPU's by about 0.5%.)"""

import numpy as np
import pytest
import torch

import paper_0909_4061_amd as rs
from oracle import adaptive, evaluate, philox
from tests.gpu_common import to_np
from workloads import build_matrix, spectrum

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _case(m, n, sigma, dtype, eps, b0, lmax, r, seed, prec="native", msd=5):
    npd = np.float32 if dtype == torch.float32 else np.float64
    A_np = build_matrix(m, n, sigma, seed=msd, dtype=npd)
    A = torch.from_numpy(A_np).to(DEV)
    print(f"tol case {m}x{n} {dtype} {prec} eps={eps} b0={b0} lmax={lmax} r={r}", flush=True)
    Q, l, est = rs.rsvd_range_finder_tol(A, eps, b0=b0, lmax=lmax, r=r, prec=prec, seed=seed)
    assert rs.device_status(DEV) & (rs.RSVD_FLAG_NONFINITE | rs.RSVD_FLAG_NOCONV) == 0
    A64 = A_np.astype(np.float64)
    Om = philox.round_to_dtype(philox.gaussian_omega(n, lmax + r, seed, 0), npd)
    ref = adaptive.blocked_adaptive_range_finder(A64, eps, r, b0, lmax, Om)
    Qg = to_np(Q).astype(np.float64)
    return dict(l=l, est=est, Q=Qg, ref=ref, A=A64, res=evaluate.residual_q(A64, Qg) if l else None)


# the oracle's estimates for this matrix after 0, 16, 32, 64, 128 columns: 23.8, 6.9, 1.6, 0.045, 1.4e-5
@pytest.mark.parametrize("eps,expect_l", [(30.0, 0), (10.0, 16), (2.0, 32), (0.1, 64), (1e-3, 128)])
def test_tol_fp64_matches_oracle(eps, expect_l):
    m, n = 700, 400
    out = _case(m, n, spectrum("exp_r", n, rate=8.0), torch.float64, eps, 16, 128, 10, seed=21)
    ref = out["ref"]
    assert out["l"] == ref["l"] == expect_l
    assert abs(out["est"] - ref["est"]) <= 1e-9 * ref["est"]
    if expect_l:
        res_ref = evaluate.residual_q(out["A"], ref["Q"])
        assert abs(out["res"] - res_ref) <= 1e-9 * res_ref
        assert out["res"] <= eps
        assert evaluate.orthonormality_error(out["Q"]) <= 1e-13


@pytest.mark.parametrize("prec", ["native", "bf16x3"])
def test_tol_fp32_matches_oracle(prec):
    m, n, eps, seed = 3000, 1500, 2e-3, 22
    sigma = spectrum("exp_r", n, rate=10.0)
    out = _case(m, n, sigma, torch.float32, eps, 16, 128, 10, seed=seed, prec=prec)
    ref = out["ref"]
    assert out["l"] == ref["l"]
    delta = 2.0 ** -24 * np.sqrt(n) if prec == "native" else 2.0 ** -16
    Om = philox.round_to_dtype(philox.gaussian_omega(n, 128 + 10, seed, 0), np.float32)
    ymax = float(np.max(np.linalg.norm(out["A"] @ Om, axis=0)))
    tol_est = 0.01 * ref["est"] + adaptive.errorest_factor() * delta * ymax
    res_ref = evaluate.residual_q(out["A"], ref["Q"])
    tol_res = 0.01 * res_ref + delta * sigma[0]
    print(f"{prec}: l {out['l']}, est {out['est']:.6e} vs oracle {ref['est']:.6e} (tol {tol_est:.2e}), "
          f"residual {out['res']:.6e} vs oracle {res_ref:.6e} (tol {tol_res:.2e})")
    assert abs(out["est"] - ref["est"]) <= tol_est
    assert abs(out["res"] - res_ref) <= tol_res
    assert out["res"] <= eps
    assert evaluate.orthonormality_error(out["Q"]) <= 1e-5


def test_tol_exact_rank_and_first_block():
    m, n, rank = 500, 300, 20
    sigma = np.zeros(n)
    sigma[:rank] = np.linspace(2.0, 1.0, rank)
    out = _case(m, n, sigma, torch.float64, 1e-8, 16, 64, 8, seed=23)
    assert out["l"] == out["ref"]["l"] == 32
    assert out["res"] <= 1e-12
    assert evaluate.orthonormality_error(out["Q"]) <= 1e-13
    # a tolerance above ||A||: the empty basis already passes
    big = _case(m, n, sigma, torch.float64, 1e3, 16, 64, 8, seed=23)
    assert big["l"] == big["ref"]["l"] == 0


def test_tol_capacity_reached():
    m, n = 600, 300
    out = _case(m, n, np.linspace(1.0, 0.5, n), torch.float64, 1e-6, 8, 32, 6, seed=24)
    assert out["l"] == out["ref"]["l"] == 32
    assert out["est"] > 1e-6 and not out["ref"]["converged"]
    assert out["res"] <= out["est"]
    assert abs(out["est"] - out["ref"]["est"]) <= 1e-9 * out["ref"]["est"]
