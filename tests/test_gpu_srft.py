"""SRFT sketch on the GPU vs the FP64 oracle, through the C ABI (marked gpu).

The GPU forms Y = A Omega, Omega = sqrt(n/l) D F_r R (Algorithm 4.5 with the
real tailoring of Section 4.6), by one FFT per row of A D.

Tolerances:
  * D and R are integer draws: identical to the oracle's.
  * Y: per row x of A, |Y_gpu - Y_oracle| <= 8 u log2(n) sqrt(2/l) ||x||_2
    entrywise (u the unit roundoff of the element type).  Every sampled DFT
    bin has magnitude of order ||x||_2; in the usual rounding model of a
    radix-2 FFT each of the log2(n) levels adds a relative error of about 2u
    (one complex multiply-add), and a factor 4 covers the pre- and
    post-processing.  A wrong index, sign or twiddle gives O(1) errors.
  * End to end: as for the Gaussian path (singular values 1e-12 / 1e-5
    relative, residual within 1e-10 / 1% of the oracle's, orthonormality).
Inputs: seeded Gaussian matrices for the sketch checks; U diag(sigma) V^T with
the recipes of workloads/ for the end-to-end checks.
"""

import math

import numpy as np
import pytest
import torch

import paper_0909_4061_amd as rs
from oracle import evaluate, philox, rsvd as orsvd
from tests.gpu_common import compare_to_oracle, to_np
from workloads import CONFIGS, build_matrix, build_matrix_torch, spectrum

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
U_OF = {torch.float64: 2.0 ** -53, torch.float32: 2.0 ** -24}


def _sketch_tol(A64, n, l, dtype):
    rown = np.linalg.norm(A64, axis=1)
    return 8.0 * U_OF[dtype] * math.log2(n) * math.sqrt(2.0 / l) * rown[:, None]


@pytest.mark.parametrize("n,l,seed,stream", [(8, 8, 1, 0), (1024, 30, 0x09094061, 0),
                                             (16384, 128, 0x09094061, 0), (4096, 128, 5, 11),
                                             (64, 64, 3, 2)])
def test_srft_draw_matches_oracle(n, l, seed, stream):
    d, R = rs.rsvd_draw_srft(n, l, 0, seed=seed, stream_id=stream, device=DEV)
    np.testing.assert_array_equal(to_np(d), philox.srft_signs(n, seed, stream))
    np.testing.assert_array_equal(to_np(R), philox.srft_sample(n, l, seed, stream))


def _sketch_case(m, n, l, lda_pad, dtype, seed):
    rng = np.random.default_rng(1000 * m + n + l)
    A_full = rng.standard_normal((m, n + lda_pad))
    A = torch.from_numpy(A_full).to(DEV, dtype)[:, :n]   # leading dimension n + lda_pad
    assert A.stride(0) == n + lda_pad
    Y = rs.rsvd_sketch(A, l, 0, sketch="srft", seed=seed)
    torch.cuda.synchronize()
    A64 = to_np(A).astype(np.float64)
    d = philox.srft_signs(n, seed)
    R = philox.srft_sample(n, l, seed)
    ref = orsvd.real_srft_sketch(A64, d, R)
    err = np.abs(to_np(Y).astype(np.float64) - ref)
    tol = _sketch_tol(A64, n, l, dtype)
    worst = float(np.max(err / tol))
    assert worst <= 1.0, f"worst error / tolerance = {worst:.3g}"
    return worst


# Every supported transform length, both load paths (even lda: paired loads; odd
# lda: element loads), ragged row counts that do not fill the persistent grid
# evenly, and l from 1 to 128.
@pytest.mark.parametrize("m,n,l,lda_pad", [
    (37, 8, 8, 0), (300, 16, 16, 0), (129, 32, 20, 0), (1000, 64, 64, 1), (257, 128, 1, 0),
    (513, 256, 128, 2), (200, 512, 77, 0), (600, 1024, 100, 1), (300, 2048, 128, 0),
    (301, 4096, 128, 3), (200, 8192, 128, 8), (3, 256, 3, 0),
])
def test_srft_sketch_fp64(m, n, l, lda_pad):
    _sketch_case(m, n, l, lda_pad, torch.float64, seed=0x09094061 + n)


@pytest.mark.parametrize("m,n,l,lda_pad", [
    (500, 16384, 128, 0), (333, 16384, 50, 1), (1111, 8192, 128, 2), (1000, 1024, 64, 1),
    (64, 64, 64, 0), (700, 4096, 128, 0), (90, 2048, 90, 5), (40, 8, 8, 0),
])
def test_srft_sketch_fp32(m, n, l, lda_pad):
    _sketch_case(m, n, l, lda_pad, torch.float32, seed=17 + n)


def test_srft_sketch_full_size_sampled_rows():
    # 32768 x 16384 FP32 (the SRFT workload's shape), l = 128, in the launch
    # configuration the benchmark times; the oracle recomputes 64 sampled rows.
    cfg = CONFIGS["srft_32768x16384"]
    sig = spectrum(cfg.spectrum, min(cfg.m, cfg.n))
    A = build_matrix_torch(cfg.m, cfg.n, sig, dtype=torch.float32, device=DEV)
    Y = rs.rsvd_sketch(A, cfg.k, cfg.p, sketch="srft", seed=cfg.m)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([[0, cfg.m - 1], np.random.default_rng(3).integers(0, cfg.m, 62)]))
    A64 = to_np(A[torch.as_tensor(rows, device=DEV)]).astype(np.float64)
    Yg = to_np(Y[torch.as_tensor(rows, device=DEV)]).astype(np.float64)
    del A, Y
    d = philox.srft_signs(cfg.n, cfg.m)
    R = philox.srft_sample(cfg.n, cfg.l, cfg.m)
    ref = orsvd.real_srft_sketch(A64, d, R)
    tol = _sketch_tol(A64, cfg.n, cfg.l, torch.float32)
    assert np.all(np.abs(Yg - ref) <= tol)


def _e2e(A64, dtype, k, p, seed):
    A = torch.from_numpy(A64).to(DEV, dtype)
    U, S, V, Q, Bt = rs.rsvd(A, k, p, 0, sketch="srft", seed=seed, return_q=True)
    torch.cuda.synchronize()
    flags = rs.device_status(DEV)
    Aread = to_np(A).astype(np.float64)
    out = compare_to_oracle(Aread, (to_np(U), to_np(S), to_np(V), to_np(Q)), k, p, 0, seed,
                            np.float64, sketch="srft")
    return out, flags


def test_srft_end_to_end_fp64():
    m, n, k, p = 2000, 1024, 20, 10
    A64 = build_matrix(m, n, spectrum("exp20", n))
    out, flags = _e2e(A64, torch.float64, k, p, seed=11)
    assert flags == 0
    assert out["sigma_rel"] <= 1e-12
    assert out["orth_q"] <= 1e-13
    assert abs(out["res_q"] - out["res_q_ref"]) <= 1e-10 * out["res_q_ref"] + 1e-14
    assert out["u_err"] <= 1e-9 and out["v_err"] <= 1e-9


def test_srft_end_to_end_fp32_gap():
    # the SRFT workload's spectrum (sigma_1..50 in [1, 2], flat 1e-3 tail) at 4096 x 2048
    m, n, k, p = 4096, 2048, 50, 78
    A64 = build_matrix(m, n, spectrum("gap", n), dtype=np.float32).astype(np.float64)
    out, flags = _e2e(A64, torch.float32, k, p, seed=12)
    assert flags == 0
    assert out["sigma_rel"] <= 1e-5
    assert out["orth_q"] <= 1e-5
    floor = 16 * U_OF[torch.float32] * out["ref"]["Sk"][0]
    assert abs(out["res_q"] - out["res_q_ref"]) <= 0.01 * out["res_q_ref"] + floor


def test_srft_matches_gaussian_quality_fp32():
    # Section 7.4 and the remarks after Theorem 11.2: in practice the SRFT sketch
    # with l = k + 20 or more does about as well as a Gaussian one.
    m, n, k, p = 3000, 1024, 40, 24
    A64 = build_matrix(m, n, spectrum("inv", n), dtype=np.float32).astype(np.float64)
    A = torch.from_numpy(A64).to(DEV, torch.float32)
    res = {}
    for sk in ("srft", "gaussian"):
        Q = rs.rsvd_range_finder(A, k, p, sketch=sk, seed=5)
        torch.cuda.synchronize()
        res[sk] = evaluate.residual_q(A64, to_np(Q).astype(np.float64))
    assert rs.device_status(DEV) == 0
    assert res["srft"] <= 2.0 * res["gaussian"]
