"""rsvd_full_static (the workspace in the library's static device array, no allocation in the
call) against rsvd_full, through the C ABI: bit for bit, since both launch the same kernels in
the same order on the same problem plan.  Two calls in a row on one device, the second with a
smaller problem (and another element type), so that the second reuses the array the first left
behind; then an oversized problem is refused before any launch."""

import ctypes

import numpy as np
import pytest
import torch

import paper_0909_4061_amd as rs
from workloads import build_matrix, spectrum

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)

CASES = [
    # (m, n, k, p, q, dtype, prec, seed): 12.4 MiB then 1.0 MiB of static workspace
    (3000, 1500, 40, 10, 1, torch.float32, "bf16x3", 21),
    (600, 300, 12, 6, 1, torch.float64, "native", 22),
]


def _matrix(m, n, dtype, seed):
    sigma = spectrum("inv", min(m, n))
    npd = np.float32 if dtype == torch.float32 else np.float64
    return torch.from_numpy(build_matrix(m, n, sigma, seed=seed, dtype=npd)).to(DEV)


def test_static_matches_rsvd_full_twice():
    for (m, n, k, p, q, dtype, prec, seed) in CASES:
        print(f"rsvd_full_static case m={m} n={n} k={k} p={p} q={q} {dtype} {prec}", flush=True)
        A = _matrix(m, n, dtype, seed)
        Us, Ss, Vs = rs.rsvd_full_static(A, k, p, q, prec=prec, seed=seed)
        Uf, Sf, Vf = rs.rsvd_full(A, k, p, q, prec=prec, seed=seed)
        torch.cuda.synchronize()
        assert rs.device_status(DEV) & ~rs.RSVD_FLAG_SHIFTED == 0
        for a, b in ((Us, Uf), (Ss, Sf), (Vs, Vf)):
            assert torch.equal(a, b)
        assert torch.all(Ss[:-1] >= Ss[1:]) and torch.all(Ss > 0)


def test_static_refuses_oversized_problem():
    # 4096 x 2048, l = 80, q = 1: rsvd_full needs 35.8 MiB > RSVD_STATIC_SCRATCH_BYTES
    A = torch.empty(4096, 2048, dtype=torch.float32, device=DEV)
    pr = rs.problem(4096, 2048, 64, 16, 1, dtype=torch.float32)
    lib = rs._lib.load()
    assert lib.rsvd_full_workspace_bytes(ctypes.byref(pr)) > rs._lib.RSVD_STATIC_SCRATCH_BYTES
    with pytest.raises(rs.RsvdError) as e:
        rs.rsvd_full_static(A, 64, 16, 1)
    assert e.value.status == rs._lib.RSVD_E_WORKSPACE
