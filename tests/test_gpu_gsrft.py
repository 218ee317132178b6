"""The Givens-chain structured test matrix on the GPU (sketch="gsrft": the remark on random Givens
rotations in Section 4.6, real form) against the oracle (oracle.gsrft) on the same A and the same
draws (signs, angles, permutations and the SRFT's D and R from (seed, stream_id); the oracle draws
them from its own generator), through the C ABI.

Tolerances.  Every stage in front of the sampler is orthogonal (the sign flips, the gathers, the two
rotation chains, the real Fourier basis), so a row of Y = A Omega has norm at most
||a_i|| sqrt(n/l) and each stage adds rounding relative to that.  A chain output out_j depends on
the rotation r < j behind it through the factor prod_{r < t < j} |s_t|, which decays geometrically
(E s^2 = 1/2 for an angle uniform on [0, 2 pi)), so the rounding of a chain, of its (cos, sin) in
the element type and of the segment scan that replaces its sequential order stays a small multiple
of u per element instead of growing with n; the FFT adds about log2(n) u.  The element test allows
(2 log2 n + 32) u ||a_i|| sqrt(n/l) per row i (u the unit roundoff of the element type); measured
at most 1.6 u ||a_i|| sqrt(n/l) over the cases (n = 8 to 16384).  The factorization built on the sketch (Algorithm 4.1 with this Omega, then
Algorithm 5.1) is compared on singular values within the FP32 / FP64 floors of the other parity
tests.
"""

import numpy as np
import pytest
import torch

import paper_0909_4061_amd as rs
from oracle import gsrft, rsvd as orsvd
from tests.gpu_common import to_np
from workloads import build_matrix

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _sketch_case(m, n, l, npd, seed, stream_id=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)).astype(npd)
    At = torch.from_numpy(A).to(DEV)
    print(f"gsrft sketch {m}x{n} l={l} {A.dtype}", flush=True)
    rs.device_status(DEV)
    Y = to_np(rs.rsvd_sketch(At, l - 2, 2, sketch="gsrft", seed=seed, stream_id=stream_id)).astype(np.float64)
    flags = rs.device_status(DEV)
    Yr = gsrft.gsrft_sketch(A.astype(np.float64), l, seed, stream_id)
    u = 2.0 ** -53 if npd == np.float64 else 2.0 ** -24
    row = np.linalg.norm(A.astype(np.float64), axis=1) * np.sqrt(n / l)
    bound = (2 * np.log2(n) + 32) * u * row
    err = np.max(np.abs(Y - Yr) / bound[:, None])
    print(f"gsrft sketch {m}x{n} l={l} {A.dtype}: max error / bound {err:.3e}")
    assert flags == 0
    return err


@pytest.mark.parametrize("m,n,l,npd", [
    (300, 256, 20, np.float64),
    (500, 1024, 24, np.float32),
    (40, 8, 5, np.float32),       # n < 256: one step per thread
    (64, 16384, 16, np.float32),  # the largest FP32 n: 64 steps per thread
    (32, 8192, 8, np.float64),    # the largest FP64 n
])
def test_gsrft_sketch_matches_oracle(m, n, l, npd):
    assert _sketch_case(m, n, l, npd, seed=31 + n) <= 1.0


def test_gsrft_stream_ids_differ():
    m, n, l = 50, 256, 10
    A = torch.from_numpy(np.random.default_rng(5).standard_normal((m, n)).astype(np.float32)).to(DEV)
    Y0 = to_np(rs.rsvd_sketch(A, l - 2, 2, sketch="gsrft", seed=7, stream_id=0))
    Y1 = to_np(rs.rsvd_sketch(A, l - 2, 2, sketch="gsrft", seed=7, stream_id=3))
    assert np.max(np.abs(Y0 - Y1)) > 1e-2
    assert _sketch_case(m, n, l, np.float32, seed=7, stream_id=3) <= 1.0


@pytest.mark.parametrize("m,n,k,p,npd", [(600, 512, 20, 10, np.float64), (2000, 1024, 30, 20, np.float32)])
def test_gsrft_rsvd_matches_oracle(m, n, k, p, npd):
    l = k + p
    sigma = np.exp(-np.arange(min(m, n)) / 8.0)
    A = build_matrix(m, n, sigma, seed=41, dtype=npd)
    A64 = A.astype(np.float64)
    print(f"gsrft rsvd {m}x{n} k={k} p={p} {A.dtype}", flush=True)
    rs.device_status(DEV)
    U, S, V = rs.rsvd(torch.from_numpy(A).to(DEV), k, p, 0, sketch="gsrft", seed=42)
    flags = rs.device_status(DEV)
    Q = gsrft.gsrft_range_finder(A64, l, 42)
    Ub, Sr, Vbt = np.linalg.svd(Q.T @ A64, full_matrices=False)
    S = to_np(S).astype(np.float64)
    u = 2.0 ** -53 if npd == np.float64 else 2.0 ** -24
    floor = (4 * np.sqrt(m) + 2 * l) * u * sigma[0]
    err = np.abs(S - Sr[:k])
    print(f"gsrft rsvd {m}x{n} {A.dtype}: max |s - ref| {err.max():.3e} (floor {floor:.3e})")
    assert flags & ~rs.RSVD_FLAG_SHIFTED == 0
    assert np.all(err <= 1e-5 * Sr[:k] + floor)
    res = np.linalg.norm(A64 - (to_np(U).astype(np.float64) * S[None, :]) @ to_np(V).astype(np.float64).T, 2)
    res_ref = np.linalg.norm(A64 - (Q @ Ub[:, :k] * Sr[None, :k]) @ Vbt[:k], 2)
    assert res <= 1.01 * res_ref + 16 * u * sigma[0], (res, res_ref)
