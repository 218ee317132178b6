"""Batched adjoint (rsvd_backward_batched, through RSVDBatchedFunction) vs the
FP64 reference gradient of oracle.rsvd_grad and vs the single-problem adjoint
(marked gpu).

Same loss and tolerance as the single-problem adjoint tests: L_i = ||U_k
diag(S_k) V_k^T - T_i||_F^2 + w_i . S_k per matrix, relative Frobenius error of
dL/dA_i within 64 l u.  Matrix i of a batch draws its test matrix from (seed,
stream_id + i).  The batches mix shapes so that problems take different
numbers of 128-column gA launches and different K splits of the adjoint's
transposed products (the recorded sequence pads them with empty steps).
"""

import numpy as np
import pytest
import torch

import paper_0909_4061_amd as rs
from oracle import philox, rsvd as orsvd
from oracle import rsvd_grad as og
from tests.gpu_common import to_np
from workloads import build_matrix, build_matrix_torch, spectrum

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
UNIT = {torch.float64: 2.0 ** -53, torch.float32: 2.0 ** -24}


@pytest.fixture(autouse=True)
def _clear_status():
    yield
    rs.device_status(DEV)


def _inputs(shapes, dtype, seed0):
    As, Ts, ws = [], [], []
    for i, (m, n, k) in enumerate(shapes):
        A64 = build_matrix(m, n, spectrum("invsqrt", min(m, n)), seed=seed0 + i,
                           dtype=np.float32 if dtype == torch.float32 else np.float64)
        rng = np.random.default_rng(seed0 + i)
        As.append(torch.from_numpy(A64).to(DEV))
        Ts.append(rng.standard_normal((m, n)))
        ws.append(rng.uniform(0.0, 1.0, k))
    return As, Ts, ws


def _batched_grads(As, Ts, ws, ks, p, q, seed, stream_id=0, prec="native"):
    leaves = [A.detach().clone().requires_grad_(True) for A in As]
    outs = rs.rsvd_batched(leaves, ks, p=p, q=q, seed=seed, stream_id=stream_id, prec=prec)
    loss = 0
    for (U, S, V), T, w, A in zip(outs, Ts, ws, As):
        Tt = torch.from_numpy(T).to(DEV, A.dtype)
        wt = torch.from_numpy(w).to(DEV, A.dtype)
        loss = loss + ((U * S[None, :]) @ V.T - Tt).square().sum() + (wt * S).sum()
    loss.backward()
    torch.cuda.synchronize()
    return [L.grad for L in leaves]


def _reference(A, k, p, q, seed, stream, T, w, dtype):
    n = A.shape[1]
    Om = philox.round_to_dtype(philox.gaussian_omega(n, k + p, seed=seed, stream=stream),
                               np.float32 if dtype == torch.float32 else np.float64)
    _, G = og.loss_and_grad(to_np(A).astype(np.float64), k, p, q, Om, T, w)
    return G


def _rel(G, Gref):
    return np.linalg.norm(to_np(G).astype(np.float64) - Gref) / np.linalg.norm(Gref)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_backward_batched_matches_reference(dtype):
    # n = 300 / 150 / 260 / 700 / 300: three, two, three, six and three gA launches;
    # m = 1200 splits the transposed products with A in the batch
    shapes = [(400, 300, 10), (200, 150, 6), (260, 260, 12), (900, 700, 20), (1200, 300, 12)]
    p, q, seed, sid = 6, 1, 11, 3
    ks = [s[2] for s in shapes]
    As, Ts, ws = _inputs(shapes, dtype, seed0=40)
    grads = _batched_grads(As, Ts, ws, ks, p, q, seed, stream_id=sid)
    for i, (A, G, T, w, k) in enumerate(zip(As, grads, Ts, ws, ks)):
        Gref = _reference(A, k, p, q, seed, sid + i, T, w, dtype)
        err = _rel(G, Gref)
        assert err <= 64.0 * (k + p) * UNIT[dtype], (i, err)
    assert rs.device_status(DEV) & ~rs.RSVD_FLAG_SHIFTED == 0


def test_backward_batched_matches_single_problem_adjoint():
    shapes = [(512, 256, 16), (333, 130, 20), (257, 257, 30)]
    p, q, seed = 8, 2, 4
    ks = [s[2] for s in shapes]
    As, Ts, ws = _inputs(shapes, torch.float32, seed0=60)
    gUs, gSs, gVs = [], [], []
    rng = np.random.default_rng(3)
    for A, k in zip(As, ks):
        m, n = A.shape
        gUs.append(torch.from_numpy(rng.standard_normal((m, k))).to(DEV, torch.float32))
        gSs.append(torch.from_numpy(rng.standard_normal(k)).to(DEV, torch.float32))
        gVs.append(torch.from_numpy(rng.standard_normal((n, k))).to(DEV, torch.float32))
    gAb = rs.rsvd_backward_batched(As, gUs, gSs, gVs, ks, p, q, seed=seed)
    torch.cuda.synchronize()
    for i, (A, k) in enumerate(zip(As, ks)):
        gA1 = rs.rsvd_backward(A, gUs[i], gSs[i], gVs[i], k, p, q, seed=seed, stream_id=i)
        torch.cuda.synchronize()
        err = float(torch.linalg.norm(gAb[i].double() - gA1.double()) / torch.linalg.norm(gA1.double()))
        assert err <= 64.0 * (k + p) * UNIT[torch.float32], (i, err)


def test_backward_batched_repoints_moved_buffers():
    # same problems and workspace, new gU / gA buffers: the recorded plan is
    # re-pointed and every call reproduces the first bit for bit; a second
    # batch in between leaves both plans usable
    shapes = [(300, 200, 10), (256, 128, 8)]
    p, q, seed = 6, 1, 2
    ks = [s[2] for s in shapes]
    As, _, _ = _inputs(shapes, torch.float64, seed0=80)
    rng = np.random.default_rng(5)
    gUs = [torch.from_numpy(rng.standard_normal((A.shape[0], k))).to(DEV) for A, k in zip(As, ks)]
    gSs = [torch.from_numpy(rng.standard_normal(k)).to(DEV) for k in ks]
    gVs = [torch.from_numpy(rng.standard_normal((A.shape[1], k))).to(DEV) for A, k in zip(As, ks)]
    probs = [rs.problem(A.shape[0], A.shape[1], k, p, q, dtype=A.dtype, seed=seed, stream_id=i)
             for i, (A, k) in enumerate(zip(As, ks))]
    arr = (rs.RsvdProblem * len(probs))(*probs)
    h = rs.handle(DEV)
    ws = torch.empty(h.lib.rsvd_backward_batched_workspace_bytes(len(probs), arr), dtype=torch.uint8, device=DEV)
    first = rs.rsvd_backward_batched(As, gUs, gSs, gVs, ks, p, q, seed=seed, ws=ws)
    torch.cuda.synchronize()
    first = [g.clone() for g in first]
    for rep in range(3):
        gU2 = [g.clone() for g in gUs]  # moved inputs
        out = [torch.full(A.shape, float("nan"), dtype=A.dtype, device=DEV) for A in As]  # moved outputs
        rs.rsvd_backward_batched(As, gU2, gSs, gVs, ks, p, q, seed=seed, ws=ws, gAs=out)
        torch.cuda.synchronize()
        for a, b in zip(out, first):
            assert torch.equal(a, b), rep
        other = [As[1][:200, :100].contiguous()]
        rs.rsvd_backward_batched(other, [gUs[1][:200].contiguous()], [gSs[1]],
                                 [gVs[1][:100].contiguous()], [ks[1]], p, q, seed=seed)
    assert rs.device_status(DEV) & ~rs.RSVD_FLAG_SHIFTED == 0


def test_backward_batched_full_size_differentiable_workload():
    # two 4096 x 2048 FP32 matrices of the differentiable workload (sigma_j =
    # j^-1/2, k = 64, p = 16, q = 1) in the bf16x3 arithmetic the benchmark
    # times; the reference gradient of the second one
    m, n, k, p, q, seed = 4096, 2048, 64, 16, 1, 5
    sig = spectrum("invsqrt", n)
    As = [build_matrix_torch(m, n, sig, seed=90 + i, dtype=torch.float32, device=DEV) for i in range(2)]
    rng = np.random.default_rng(90)
    Ts = [rng.standard_normal((m, n)) for _ in range(2)]
    ws = [rng.uniform(0.0, 1.0, k) for _ in range(2)]
    grads = _batched_grads(As, Ts, ws, [k, k], p, q, seed, prec="bf16x3")
    Gref = _reference(As[1], k, p, q, seed, 1, Ts[1], ws[1], torch.float32)
    err = _rel(grads[1], Gref)
    print(f"batched backward bf16x3 {m}x{n} k={k}: rel err {err:.3e} ({err / (k + p) / 2.0 ** -16:.3f} l 2^-16)")
    # bf16x3 products: x = hi + lo carries a relative error up to 2^-16 per element; the bound is
    # the one of the single-matrix adjoint tests, 2 l 2^-16 (measured here: 0.013 l 2^-16)
    assert err <= 2.0 * (k + p) * 2.0 ** -16, err


def test_backward_batched_kept_matches_recomputation():
    # the kept batched adjoint returns the recomputing adjoint's gA, bit for bit; the
    # kept batched forward (CholeskyQR2 for every basis) returns rsvd_batched's outputs
    # (one pass for the bases inside the power scheme) up to FP32 rounding
    shapes = [(400, 300, 10), (200, 150, 6), (900, 700, 20)]
    p, q, seed = 6, 1, 8
    ks = [s[2] for s in shapes]
    As, _, _ = _inputs(shapes, torch.float32, seed0=120)
    rng = np.random.default_rng(8)
    gUs = [torch.from_numpy(rng.standard_normal((A.shape[0], k))).to(DEV, torch.float32) for A, k in zip(As, ks)]
    gSs = [torch.from_numpy(rng.standard_normal(k)).to(DEV, torch.float32) for k in ks]
    gVs = [torch.from_numpy(rng.standard_normal((A.shape[1], k))).to(DEV, torch.float32) for A, k in zip(As, ks)]
    ref = rs.rsvd_batched(As, ks, p=p, q=q, seed=seed)
    outs, ws = rs.rsvd_batched_kept(As, ks, p, q, seed=seed)
    g_re = rs.rsvd_backward_batched(As, gUs, gSs, gVs, ks, p, q, seed=seed)
    g_kept = rs.rsvd_backward_batched_kept(As, gUs, gSs, gVs, ks, p, q, ws, seed=seed)
    torch.cuda.synchronize()
    for (U, S, V), (U0, S0, V0) in zip(outs, ref):
        S, S0 = S.double().cpu().numpy(), S0.double().cpu().numpy()
        assert np.max(np.abs(S - S0) / S0) <= 1e-5
        Uk, Vk = orsvd.normalize_signs(U.double().cpu().numpy(), V.double().cpu().numpy())
        U0, V0 = orsvd.normalize_signs(U0.double().cpu().numpy(), V0.double().cpu().numpy())
        assert max(np.max(np.abs(Uk - U0)), np.max(np.abs(Vk - V0))) <= 1e-3
    for a, b in zip(g_kept, g_re):
        assert torch.equal(a, b)
