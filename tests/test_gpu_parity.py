"""GPU path vs the FP64 CPU oracle, through the C ABI (marked gpu).

Tolerances (element type FP64 / FP32):
  * test matrix Omega: FP64 entries within 8 ulp of the oracle's (device and host
    log/cos differ in the last bits); FP32 entries identical except for values
    whose FP64 draw lies within those ulps of an FP32 rounding boundary;
  * singular values: relative error <= 1e-12 (FP64) / 1e-5 (FP32, the stated
    budget) for the k retained values;
  * residual ||A - QQ*A||_2 of the GPU basis within 1e-10 (FP64) / 1% (FP32)
    of the oracle basis's residual, with a floor of 16 u sigma_1 (u the unit
    roundoff of the element type): a basis stored in FP32 cannot resolve a
    residual below its own rounding, e.g. when l = min(m, n) and the exact
    residual is zero;
  * orthonormality max|Q*Q - I| <= 1e-13 (FP64) / 1e-5 (FP32).
Inputs are seeded U diag(sigma) V^T matrices from workloads/.
"""

import numpy as np
import pytest
import torch

import paper_0909_4061_amd as rs
from oracle import evaluate, philox, rsvd as orsvd
from tests.gpu_common import compare_to_oracle, to_np
from workloads import build_matrix, spectrum

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _run(A, k, p, q, seed=0, prec="native", stream_id=0):
    U, S, V, Q, Bt = rs.rsvd(A, k, p, q, seed=seed, prec=prec, stream_id=stream_id, return_q=True)
    torch.cuda.synchronize()
    flags = rs.device_status(DEV)
    return (to_np(U), to_np(S), to_np(V), to_np(Q)), flags, Bt


@pytest.mark.parametrize("n,l", [(1000, 30), (8192, 120), (37, 5), (1, 1)])
def test_omega_fp64_matches_oracle(n, l):
    seed = 0x09094061
    om = to_np(rs.rsvd_draw_omega(n, l, 0, dtype=torch.float64, seed=seed, device=DEV))
    ref = philox.gaussian_omega(n, l, seed=seed)
    ulp = np.spacing(np.abs(ref))
    assert np.all(np.abs(om - ref) <= 8 * ulp)


def test_omega_fp32_matches_oracle():
    seed = 77
    n, l = 8192, 120
    om = to_np(rs.rsvd_draw_omega(n, l, 0, dtype=torch.float32, seed=seed, device=DEV, stream_id=3))
    ref64 = philox.gaussian_omega(n, l, seed=seed, stream=3)
    ref = ref64.astype(np.float32)
    mism = np.argwhere(om != ref)
    # any mismatch must be a one-ulp rounding-boundary case
    for i, j in mism:
        assert abs(float(om[i, j]) - float(ref[i, j])) <= np.spacing(np.float32(abs(ref[i, j]))) * 1.0001
    assert len(mism) <= 4


# The Gram of one call is split into row chunks x groups of 16 x 16 tiles: (40000, 100) uses
# 512-row chunks (8 stages) and three tile groups with a 64-row last chunk; (20001, 64) uses
# 128-row chunks, one tile group and a 33-row last chunk.  FP32 Q = Y R^-1 runs in place on the
# short-product kernel (32-row blocks, all of K = l in registers): 16-byte row loads when
# l % 8 == 0 (120, 64, 128, 96), element loads otherwise (100, 45, 33, 7, 1); odd l leaves the
# second K half one short (33, 7, 45, 1); l <= 32 / <= 64 / <= 128 take the three register
# sizes; l <= 96 leaves waves without columns; 24 rows are fewer than one block.
@pytest.mark.parametrize("dtype,rows,l", [(torch.float64, 2000, 30), (torch.float32, 5000, 120),
                                          (torch.float32, 333, 45), (torch.float64, 129, 128),
                                          (torch.float32, 64, 1), (torch.float32, 40000, 100),
                                          (torch.float32, 20001, 64), (torch.float32, 1001, 7),
                                          (torch.float32, 517, 33), (torch.float32, 300, 128),
                                          (torch.float32, 1001, 96), (torch.float32, 24, 24)])
def test_cholesky_qr2_matches_householder(dtype, rows, l):
    rng = np.random.default_rng(rows + l)
    Y64 = rng.standard_normal((rows, l)) @ np.diag(np.linspace(1.0, 0.05, l))
    Y = torch.from_numpy(Y64).to(DEV, dtype)
    Yin = to_np(Y).astype(np.float64)
    Q, R = rs.rsvd_orth(Y.clone())
    torch.cuda.synchronize()
    assert rs.device_status(DEV) == 0
    Qo, Ro = orsvd.qr_pos(Yin)
    tol = 1e-12 if dtype == torch.float64 else 2e-5
    assert np.max(np.abs(to_np(Q) - Qo)) < tol * 10
    assert np.max(np.abs(to_np(R) - Ro)) < tol * 10 * np.max(np.abs(Ro))
    assert evaluate.orthonormality_error(to_np(Q).astype(np.float64)) < (1e-13 if dtype == torch.float64 else 1e-5)


def test_c1_fp64_end_to_end():
    # 2000 x 1000, sigma_j = exp(-j/20), k = 20, p = 10, q = 0, Gaussian Omega.
    m, n, k, p, q = 2000, 1000, 20, 10, 0
    sigma = spectrum("exp20", n)
    A64 = build_matrix(m, n, sigma, seed=0x09094061)
    A = torch.from_numpy(A64).to(DEV)
    out, flags, _ = _run(A, k, p, q, seed=0x09094061)
    assert flags == 0
    r = compare_to_oracle(A64, out, k, p, q, 0x09094061, np.float64)
    assert r["sigma_rel"] <= 1e-12
    assert abs(r["res_q"] - r["res_q_ref"]) <= 1e-10 * r["res_q_ref"]
    assert r["orth_q"] <= 1e-13
    assert r["u_err"] < 1e-9 and r["v_err"] < 1e-9
    # the residual sits between sigma_{l+1} (Mirsky) and the Cor 10.9 bound
    assert sigma[k + p] * (1 - 1e-9) <= r["res_q"] <= evaluate.cor10_9_bound(sigma, k, p)


# l = k + p spans every compiled Jacobi size: 30 (<= 32), 45 (<= 64), 80 (<= 96), 128.
@pytest.mark.parametrize("m,n,k,p,q", [(2048, 1024, 20, 10, 2), (1000, 333, 30, 15, 1), (300, 257, 1, 0, 0),
                                       (130, 128, 100, 28, 1), (1500, 700, 70, 10, 1)])
def test_fp32_power_iteration_parity(m, n, k, p, q):
    sigma = spectrum("inv", min(m, n))
    A32 = build_matrix(m, n, sigma, seed=m + n, dtype=np.float32)
    A64 = A32.astype(np.float64)
    A = torch.from_numpy(A32).to(DEV)
    out, flags, _ = _run(A, k, p, q, seed=9)
    r = compare_to_oracle(A64, out, k, p, q, 9, np.float32)
    assert r["sigma_rel"] <= 1e-5, r["sigma_rel"]
    floor = 16 * np.finfo(np.float32).eps / 2 * sigma[0]
    assert abs(r["res_q"] - r["res_q_ref"]) <= 0.01 * r["res_q_ref"] + floor
    assert abs(r["res_k"] - r["res_k_ref"]) <= 0.01 * r["res_k_ref"] + floor
    assert r["orth_q"] <= 1e-5
    assert flags & ~rs.RSVD_FLAG_SHIFTED == 0


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
def test_bf16_paths_residual(prec):
    m, n, k, p, q = 2048, 1024, 20, 10, 2
    sigma = spectrum("inv", n)
    A32 = build_matrix(m, n, sigma, seed=5, dtype=np.float32)
    A64 = A32.astype(np.float64)
    A = torch.from_numpy(A32).to(DEV)
    out32, _, _ = _run(A, k, p, q, seed=3)
    outb, _, _ = _run(A, k, p, q, seed=3, prec=prec)
    res32 = evaluate.residual_usv(A64, out32[0].astype(np.float64), out32[1].astype(np.float64),
                                  out32[2].astype(np.float64))
    resb = evaluate.residual_usv(A64, outb[0].astype(np.float64), outb[1].astype(np.float64),
                                 outb[2].astype(np.float64))
    sig_err = np.max(np.abs(outb[1] - out32[1]) / out32[1])
    if prec == "bf16x3":
        assert abs(resb - res32) <= 0.01 * res32, (resb, res32)
        assert sig_err < 1e-3
    else:
        assert resb <= 1.5 * res32  # plain BF16: coarse, but still a valid low-rank approximation
    assert evaluate.orthonormality_error(outb[3].astype(np.float64)) <= 1e-5


def test_deterministic():
    m, n, k, p, q = 3000, 1500, 40, 10, 1
    sigma = spectrum("inv", n)
    A = torch.from_numpy(build_matrix(m, n, sigma, seed=1, dtype=np.float32)).to(DEV)
    a, _, _ = _run(A, k, p, q, seed=4)
    b, _, _ = _run(A, k, p, q, seed=4)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_exact_rank_uses_shift():
    # rank 5 < l = 12: Y has 7 roundoff-level singular values; CholeskyQR needs a shift.
    m, n, rank = 500, 200, 5
    sigma = np.zeros(n)
    sigma[:rank] = [5, 3, 2, 1, 0.5]
    A64 = build_matrix(m, n, sigma, seed=3)
    A = torch.from_numpy(A64).to(DEV)
    out, flags, _ = _run(A, rank, 7, 1, seed=2)
    assert flags & rs.RSVD_FLAG_SHIFTED
    assert np.max(np.abs(out[1] - sigma[:rank]) / sigma[:rank]) < 1e-7
    assert evaluate.orthonormality_error(out[3]) < 1e-10
    assert evaluate.residual_usv(A64, *out[:3]) < 1e-7


@pytest.mark.parametrize("prec", ["native", "bf16x3"])
@pytest.mark.parametrize("kind", ["exact_rank", "steep"])
def test_fp32_shifted_inner_bases_match_oracle(kind, prec):
    # FP32 data whose sketches are numerically rank deficient (exact rank 6 < l = 16, or a spectrum
    # falling below FP32 resolution within l), so that CholeskyQR needs the shift in the inner bases
    # of the power scheme and in the final one.  Against the oracle (Householder QR at every step): singular values within 1e-5
    # relative plus the FP32 floor (4 sqrt(m) + 2 l) u sigma_1 (2^-16 sigma_1 for bf16x3 products),
    # the residual within 1% of the oracle's plus that floor, orthonormal U and Q.
    m, n, k, p, q = 1500, 600, 6, 10, 2
    if kind == "exact_rank":
        sigma = np.zeros(n)
        sigma[:k] = [4.0, 3.0, 2.0, 1.5, 1.0, 0.5]
    else:
        sigma = spectrum("exp_r", n, rate=0.5)  # sigma_16 / sigma_1 = e^-30: below FP32 resolution
    A32 = build_matrix(m, n, sigma, seed=11, dtype=np.float32)
    A64 = A32.astype(np.float64)
    A = torch.from_numpy(A32).to(DEV)
    out, flags, _ = _run(A, k, p, q, seed=6, prec=prec)
    if kind == "exact_rank":
        assert flags & rs.RSVD_FLAG_SHIFTED
    assert flags & ~rs.RSVD_FLAG_SHIFTED == 0
    r = compare_to_oracle(A64, out, k, p, q, 6, np.float32)
    ref = r["ref"]
    u = 2.0 ** -24 if prec == "native" else 2.0 ** -16
    floor = (4.0 * np.sqrt(m) + 2.0 * (k + p)) * u * ref["Sk"][0]
    err = np.abs(out[1].astype(np.float64) - ref["Sk"])
    print(f"{kind} {prec}: max sigma err / (1e-5 sigma + floor) "
          f"{np.max(err / (1e-5 * ref['Sk'] + floor)):.3f}, residual {r['res_k']:.3e} vs {r['res_k_ref']:.3e}")
    assert np.all(err <= 1e-5 * ref["Sk"] + floor)
    assert abs(r["res_k"] - r["res_k_ref"]) <= 0.01 * r["res_k_ref"] + floor
    assert evaluate.orthonormality_error(out[0].astype(np.float64)) <= 1e-5
    assert r["orth_q"] <= 1e-5


def test_strided_rows():
    # lda > n: a column slice of a wider matrix
    m, n, k, p = 700, 300, 10, 5
    sigma = spectrum("exp_r", n, rate=10.0)
    A64 = build_matrix(m, n, sigma, seed=8)
    wide = np.zeros((m, n + 7))
    wide[:, :n] = A64
    W = torch.from_numpy(wide).to(DEV)
    out, flags, _ = _run(W[:, :n], k, p, 1, seed=1)
    r = compare_to_oracle(A64, out, k, p, 1, 1, np.float64)
    assert r["sigma_rel"] <= 1e-12 and flags == 0


@pytest.mark.parametrize("prec", ["native", "bf16x3"])
def test_strided_rows_fp32(prec):
    # lda = n + 7 is not a multiple of four: the streaming GEMMs take their scalar-load path
    m, n, k, p, q = 1500, 700, 24, 8, 1
    sigma = spectrum("inv", n)
    A32 = build_matrix(m, n, sigma, seed=12, dtype=np.float32)
    wide = np.zeros((m, n + 7), dtype=np.float32)
    wide[:, :n] = A32
    W = torch.from_numpy(wide).to(DEV)
    out, flags, _ = _run(W[:, :n], k, p, q, seed=6, prec=prec)
    dense = torch.from_numpy(A32).to(DEV)
    ref_out, _, _ = _run(dense, k, p, q, seed=6, prec=prec)
    # same arithmetic, same order: identical results whatever the leading dimension
    for x, y in zip(out, ref_out):
        assert np.array_equal(x, y)
    if prec == "native":
        r = compare_to_oracle(A32.astype(np.float64), out, k, p, q, 6, np.float32)
        assert r["sigma_rel"] <= 1e-5
