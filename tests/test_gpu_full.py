"""rsvd_full (the four hot-path calls as one, replayed from a HIP graph) vs the
four separate calls on the same inputs (marked gpu).

The graph holds the same launches in the same order, so every replay must
reproduce the separate calls bit for bit.  Each case replays the graph
several times with eager work and synchronizations in between, clears the
outputs before each replay, and finally decomposes new contents of A in the
same buffer (sigma scales with A).
"""

import numpy as np
import pytest
import torch

import paper_0909_4061_amd as rs
from workloads import build_matrix, spectrum

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


@pytest.fixture(autouse=True)
def _clear_status():
    yield
    rs.device_status(DEV)


@pytest.mark.parametrize("m,n,k,p,q,dtype,prec,sketch", [
    (2000, 1000, 20, 10, 0, torch.float64, "native", "gaussian"),   # the FP64 latency-scale problem
    (1500, 700, 70, 10, 2, torch.float32, "bf16x3", "gaussian"),    # split K, power steps, l = 80
    (333, 130, 20, 12, 1, torch.float32, "native", "gaussian"),     # ragged tiles
    (600, 512, 30, 18, 0, torch.float32, "bf16x3", "srft"),         # SRFT sketch
])
def test_full_replays_match_separate_calls(m, n, k, p, q, dtype, prec, sketch):
    A64 = build_matrix(m, n, spectrum("exp_r", min(m, n), rate=12.0), seed=m + n,
                       dtype=np.float32 if dtype == torch.float32 else np.float64)
    A = torch.from_numpy(A64).to(DEV)
    ref = rs.rsvd(A, k, p, q, sketch=sketch, prec=prec, seed=7)
    pr = rs.problem(m, n, k, p, q, dtype=dtype, sketch=sketch, prec=prec, seed=7)
    ws = rs.full_workspace(pr, DEV)
    outs = rs.rsvd_full(A, k, p, q, sketch=sketch, prec=prec, seed=7, ws=ws)   # captures
    torch.cuda.synchronize()
    for rep in range(3):
        for t in outs:
            t.fill_(float("nan"))
        junk = torch.randn(256, 256, device=DEV) @ torch.randn(256, 256, device=DEV)  # eager work between replays
        torch.cuda.synchronize()
        rs.rsvd_full(A, k, p, q, sketch=sketch, prec=prec, seed=7, outs=outs, ws=ws)  # replays
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a, b), rep
        del junk
    A.mul_(2.0)
    rs.rsvd_full(A, k, p, q, sketch=sketch, prec=prec, seed=7, outs=outs, ws=ws)
    torch.cuda.synchronize()
    np.testing.assert_allclose(outs[1].double().cpu().numpy(), 2.0 * ref[1].double().cpu().numpy(),
                               rtol=1e-5 if dtype == torch.float32 else 1e-12)
    assert rs.device_status(DEV) & ~rs.RSVD_FLAG_SHIFTED == 0
