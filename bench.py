"""Benchmark of the randomized SVD hot path on one MI355X.

One step = the whole path on the resident input: draw Omega, Y = A Omega,
CholeskyQR2, q power steps (A^T Q, CQR2, A Qt, CQR2), B = Q* A, the FP64 small
SVD and the lifts -- the four C entry points rsvd_range_finder,
rsvd_power_iter, rsvd_project and rsvd_svd.

Workload (default): power-iteration rSVD of an FP32 16384 x 8192 matrix
A = U diag(sigma) V^T with sigma_j = 1/j (U, V Haar, built on the GPU), k = 100,
p = 20, q = 2.  The headline line is the BF16-MFMA form (bf16x3 split products,
FP32 accumulation); the plain FP32 form runs on the same matrix for comparison.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.  `value` is algorithmic TFLOP/s of the whole step
(flops the method must do, not padded tiles or the three bf16 products).
The default run also times the two-sided single pass (Section 5.5) against the
two-pass route with q = 0 on the same matrix ("single_pass_two_sided"), and the
other workloads briefly (FP64 2000 x 1000; the SRFT workload, FP32
32768 x 16384, with the SRFT, Gaussian and Givens-chain test matrices; 512
uneven matrices; 32 differentiable 4096 x 2048 matrices; Stage B of a psd
16384 x 16384 matrix) and reports them compactly under "workloads"; each has
its own --workload mode with a full line.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the streaming GEMMs (scaled FETCH_SIZE + WRITE_SIZE from rocprofv3
# counter runs, profiles/stream_gemm_power_iteration_16384x8192_hbm_counters.md), valid only for
# the kernel source they were measured on and the 16384 x 8192, l = 120 shape.
# (The FP32-product kernels were not counted for this source: their traffic is reported as null.)
TRAFFIC_KERNEL_SHA = "c2f37a66479cb19d"
TRAFFIC_SHAPE = (16384, 8192, 120)
TRAFFIC_BYTES = {"stream_tn_bf16x3": 583809978, "stream_nn_bf16x3": 579173204}
# The same for the SRFT row-FFT kernel at 32768 x 16384, l = 128
# (profiles/srft_sketch_32768x16384_hbm_counters.md).
SRFT_TRAFFIC_SHA = "2b16782d46e9052b"
SRFT_TRAFFIC_SHAPE = (32768, 16384, 128)
SRFT_TRAFFIC_BYTES = 2165559296
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "f64": 78.6}
MI355X_CUS = 256


def algorithmic_flops(m, n, l, k, q):
    """Flops the method must do per step.

    GEMM passes over A: (2q + 2) x 2 m n l.  A QR factorization of an M x l
    matrix: 2 M l^2 (Householder's 2 M l^2 - 2 l^3 / 3, rounded up; how many
    CholeskyQR passes the implementation takes is not counted).  QRs: one of m
    rows, then n and m rows per power step.  Small SVD: Gram of Bt n l^2
    (+ O(l^3)).  Lifts: 2 (m + n) l k.
    """
    gemm = (2 * q + 2) * 2.0 * m * n * l
    qr = 2.0 * l * l * (m + q * (m + n))
    small = n * l * l + 2.0 * (m + n) * l * k
    return gemm + qr + small


def e2e_floor(m, n, l, k, q, prec, esize=4):
    """The step's roofline floor: the larger of its algorithmic HBM bytes at 8 TB/s and its
    GEMM flops at the peak of the arithmetic that streams A (bf16x3: three BF16 products)."""
    hbm_ms = algorithmic_bytes(m, n, l, q, esize) / (PEAK_HBM_GBS * 1e9) * 1e3
    gemm = (2 * q + 2) * 2.0 * m * n * l
    if prec == "native":
        mf_ms = gemm / (PEAK_TFLOPS["f64" if esize == 8 else "f32"] * 1e12) * 1e3
    else:
        mf_ms = (3 if prec == "bf16x3" else 1) * gemm / (PEAK_TFLOPS["bf16"] * 1e12) * 1e3
    bound = "hbm" if hbm_ms >= mf_ms else "mfma"
    return {"bound": bound, "floor_ms": max(hbm_ms, mf_ms), "hbm_floor_ms": hbm_ms, "mfma_floor_ms": mf_ms}


def algorithmic_bytes(m, n, l, q, esize=4):
    """HBM bytes the method must move per step: every pass reads A once and its
    l-column operand, and writes its l-column result."""
    return (2 * q + 2) * (m * n + (m + n) * l) * esize


def spectral_norm_residual(A, U, S, V, iters=40, block=32, seed=1234):
    """||A - U diag(S) V^T||_2 in FP64 by block subspace iteration with a final
    Rayleigh-Ritz step (torch on the GPU; a measurement, not part of the method).
    40 iterations of a 32-column block agree with the dense-SVD norm to 2e-8
    relative even when the residual's leading singular values form a flat
    cluster (tests/test_evaluator.py); 30 x 16 left 9e-5 there."""
    import torch
    A64 = A.double()
    U64, S64, V64 = U.double(), S.double(), V.double()
    gen = torch.Generator(device=A.device)
    gen.manual_seed(seed)
    X = torch.randn(A.shape[1], block, generator=gen, device=A.device, dtype=torch.float64)

    def E(x):
        return A64 @ x - U64 @ (S64[:, None] * (V64.T @ x))

    def Et(y):
        return A64.T @ y - V64 @ (S64[:, None] * (U64.T @ y))

    for _ in range(iters):
        X, _ = torch.linalg.qr(Et(E(X)))
    s = torch.linalg.svdvals(E(X))
    out = float(s[0])
    del A64
    return out


def run_path(A, k, p, q, prec, steps, warmup, seed):
    import torch
    import paper_0909_4061_amd as rs

    m, n = A.shape
    l = k + p
    dev = A.device
    pr = rs.problem(m, n, k, p, q, dtype=A.dtype, prec=prec, seed=seed, lda=A.stride(0))
    ws = rs.Workspace(pr, dev)
    Q = torch.empty(m, l, dtype=A.dtype, device=dev)
    Bt = torch.empty(n, l, dtype=A.dtype, device=dev)
    U = torch.empty(m, k, dtype=A.dtype, device=dev)
    S = torch.empty(k, dtype=A.dtype, device=dev)
    V = torch.empty(n, k, dtype=A.dtype, device=dev)
    kw = dict(prec=prec, seed=seed, ws=ws)

    def step():
        rs.rsvd_range_finder(A, k, p, q=q, Q=Q, **kw)
        rs.rsvd_power_iter(A, Q, k, p, q, **kw)
        rs.rsvd_project(A, Q, k, p, q=q, Bt=Bt, **kw)
        rs.rsvd_svd(Bt, Q, m, n, k, p, q=q, dtype=A.dtype, U=U, S=S, V=V, **kw)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # Timed region: HIP events bracket only the launches of the streaming GEMMs
    # (the roofline kernel), so the step time carries few extra events.
    rs.profile_enable(16 * max(steps, 1), dev)
    rs.profile_select(["stream_nn", "stream_tn"], dev)
    stream = torch.cuda.current_stream(dev)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    ms_total = t0.elapsed_time(t1)
    prof = rs.profile_read(dev)
    # Per-family breakdown in separate steps with every launch bracketed.
    nb = 2
    rs.profile_enable(128 * nb, dev)
    for _ in range(nb):
        step()
    breakdown = {f: v[1] / nb for f, v in rs.profile_read(dev).items()}
    rs.profile_enable(0, dev)
    flags = rs.device_status(dev)
    return dict(ms_per_step=ms_total / steps, prof=prof, breakdown=breakdown, flags=flags, U=U, S=S, V=V)


def single_pass_general(A, k, p, sigma, prec, steps, warmup, seed):
    """The two-sided single pass of Section 5.5 (rsvd_svd_onepass: Y = A Omega and Yt = A^T Omegat,
    the core from its two least-squares relations) against the two-pass route it replaces (range
    finder with q = 0, B = Q^T A, small SVD), each timed end to end on the same A."""
    import torch
    import paper_0909_4061_amd as rs

    m, n = A.shape
    l = k + p
    dev = A.device
    pr = rs.problem(m, n, k, p, 0, dtype=A.dtype, prec=prec, seed=seed, lda=A.stride(0))
    ws = rs.Workspace(pr, dev)
    Q = torch.empty(m, l, dtype=A.dtype, device=dev)
    Bt = torch.empty(n, l, dtype=A.dtype, device=dev)
    U = torch.empty(m, k, dtype=A.dtype, device=dev)
    S = torch.empty(k, dtype=A.dtype, device=dev)
    V = torch.empty(n, k, dtype=A.dtype, device=dev)
    kw = dict(prec=prec, seed=seed, ws=ws)

    def one_pass():
        rs.rsvd_svd_onepass(A, k, p, U=U, S=S, V=V, **kw)

    def two_pass():
        rs.rsvd_range_finder(A, k, p, Q=Q, **kw)
        rs.rsvd_project(A, Q, k, p, Bt=Bt, **kw)
        rs.rsvd_svd(Bt, Q, m, n, k, p, dtype=A.dtype, U=U, S=S, V=V, **kw)

    stream = torch.cuda.current_stream(dev)
    out = {}
    for name, fn in (("onepass", one_pass), ("twopass_q0", two_pass)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        rs.device_status(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        flags = rs.device_status(dev)
        err = spectral_norm_residual(A, U, S, V) / sigma[k]
        out[name] = {"ms_per_call": ms, "passes_over_a": 1 if name == "onepass" else 2, "err_ratio": err,
                     "flags": flags}
        print(f"# general single pass {prec} {name}: {ms:.3f} ms per call, err ratio {err:.4f}",
              file=sys.stderr, flush=True)
    del ws
    return out


def srft_flops(m, n, l, k):
    """Flops of the SRFT rSVD per step: the real FFT of every row (2.5 n log2 n
    each, the usual count for a length-n real transform), CholeskyQR2 of Y
    (4 m l^2), the projection 2 m n l, the small SVD's Gram n l^2 and the lifts."""
    import math
    return 2.5 * m * n * math.log2(n) + 4.0 * m * l * l + 2.0 * m * n * l + n * l * l + 2.0 * (m + n) * l * k


def run_srft_workload(A, k, p, prec, steps, warmup, seed):
    """Stage A alone and the whole rSVD, with the SRFT and with the Gaussian test matrix."""
    import torch
    import paper_0909_4061_amd as rs

    m, n = A.shape
    l = k + p
    dev = A.device
    Q = torch.empty(m, l, dtype=A.dtype, device=dev)
    Bt = torch.empty(n, l, dtype=A.dtype, device=dev)
    U = torch.empty(m, k, dtype=A.dtype, device=dev)
    S = torch.empty(k, dtype=A.dtype, device=dev)
    V = torch.empty(n, k, dtype=A.dtype, device=dev)
    stream = torch.cuda.current_stream(dev)
    out = {}
    for sketch in ("srft", "gaussian", "gsrft"):
        pr = rs.problem(m, n, k, p, 0, dtype=A.dtype, sketch=sketch, prec=prec, seed=seed, lda=A.stride(0))
        ws = rs.Workspace(pr, dev)
        kw = dict(sketch=sketch, prec=prec, seed=seed, ws=ws)

        def stage_a():
            rs.rsvd_range_finder(A, k, p, Q=Q, **kw)

        def stage_b():
            rs.rsvd_project(A, Q, k, p, Bt=Bt, **kw)
            rs.rsvd_svd(Bt, Q, m, n, k, p, dtype=A.dtype, U=U, S=S, V=V, **kw)

        for _ in range(warmup):
            stage_a()
            stage_b()
        torch.cuda.synchronize()
        rs.profile_enable(16 * max(steps, 1), dev)
        rs.profile_select(["srft", "gsrft", "stream_nn", "stream_tn"], dev)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps + 1)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for i in range(steps):
            stage_a()
            ev[2 * i + 1].record(stream)
            stage_b()
            ev[2 * i + 2].record(stream)
        torch.cuda.synchronize()
        a_ms = sum(ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(steps)) / steps
        total_ms = ev[0].elapsed_time(ev[-1]) / steps
        prof = rs.profile_read(dev)
        rs.profile_enable(128 * 2, dev)
        for _ in range(2):
            stage_a()
            stage_b()
        breakdown = {f: v[1] / 2 for f, v in rs.profile_read(dev).items()}
        rs.profile_enable(0, dev)
        flags = rs.device_status(dev)
        out[sketch] = dict(ms_per_step=total_ms, stage_a_ms=a_ms, prof=prof, breakdown=breakdown, flags=flags,
                           U=U.clone(), S=S.clone(), V=V.clone())
        del ws
    return out


def srft_roofline(res, m, n, l):
    import hashlib
    launches, total_ms = res["prof"]["srft"]
    avg_s = total_ms / launches / 1e3
    bytes_launch = 4.0 * m * n + 4.0 * m * l + 8.0 * n + 4.0 * l
    achieved = bytes_launch / avg_s / 1e9
    src = os.path.join(ROOT, "paper_0909_4061_amd", "csrc", "k_srft.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    traffic = SRFT_TRAFFIC_BYTES if (sha == SRFT_TRAFFIC_SHA and (m, n, l) == SRFT_TRAFFIC_SHAPE) else None
    return {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "kernel": "srft_rows_f32",
            "launches": launches, "avg_us": avg_s * 1e6, "per_launch": {"bytes": bytes_launch}}


def workload_srft(args, A, sigma):
    import numpy as np
    m, n = A.shape
    k, p = args.k, args.p
    l = k + p
    res = run_srft_workload(A, k, p, args.srft_prec, args.steps, args.warmup, args.seed)
    gflops = 2.0 * m * n * l * 2 + 4.0 * m * l * l + n * l * l + 2.0 * (m + n) * l * k
    paths = {}
    for sk, r in res.items():
        err = spectral_norm_residual(A, r["U"], r["S"], r["V"]) / sigma[k]
        sig_err = float(np.max(np.abs(r["S"].double().cpu().numpy() - sigma[:k]) / sigma[:k]))
        fl = srft_flops(m, n, l, k) if sk != "gaussian" else gflops
        s = r["ms_per_step"] / 1e3
        paths[sk] = {"ms_per_step": r["ms_per_step"], "stage_a_ms": r["stage_a_ms"], "tflops": fl / s / 1e12,
                     "a_read_gbs_stage_a": 4.0 * m * n / (r["stage_a_ms"] / 1e3) / 1e9,
                     "err_ratio": err, "sigma_rel_err_vs_construction": sig_err, "flags": r["flags"],
                     "kernel_ms_per_step": r["breakdown"]}
        print(f"# {sk}: {r['ms_per_step']:.3f} ms/step (stage A {r['stage_a_ms']:.3f} ms), err ratio {err:.4f}",
              file=sys.stderr, flush=True)
    hp = paths["srft"]
    line = {
        "metric": "rSVD TFLOP/s + HBM GB/s at stated ||A-USV*||/sigma_{k+1}; SRFT vs Gaussian sketch",
        "value": hp["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": hp["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "prec": args.srft_prec, "data": "synthetic",
        "config": {"workload": f"SRFT vs Gaussian sketch rSVD, FP32 {m}x{n}, spectral gap, k={k}, p={p}, q=0",
                   "m": m, "n": n, "k": k, "p": p, "q": 0, "sketch": "srft"},
        "err_ratio": hp["err_ratio"], "roofline": srft_roofline(res["srft"], m, n, l),
        "stage_a_speedup_vs_gaussian": paths["gaussian"]["stage_a_ms"] / hp["stage_a_ms"],
        "gsrft_pretransform": gsrft_roofline(res["gsrft"], m, n),
        "paths": paths,
    }
    return line


def gsrft_roofline(res, m, n):
    """The Givens-chain pretransform kernel: A read once and its transformed copy written once
    (8 m n bytes for FP32; the tables, 72 n bytes, are read from L2 by every row)."""
    launches, total_ms = res["prof"]["gsrft"]
    avg_s = total_ms / launches / 1e3
    bytes_launch = 8.0 * m * n
    achieved = bytes_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": None, "kernel": "gsrft_rows_f32", "launches": launches,
            "avg_us": avg_s * 1e6, "per_launch": {"bytes": bytes_launch}}


def workload_psd(args):
    """Stage B for a positive semidefinite A (Algorithm 5.3 direct eigendecomposition, Algorithm 5.5
    Nystrom) on an FP32 16384 x 16384 matrix: A = V diag(lam) V^T + 1e-4 I with lam_j = 1/j for
    j <= 4096 (V a thin Haar basis), k = 100, p = 20, Q from the range finder with q = 1.  Each
    Stage B call reads A once (the product A Q); it is timed alone, with its A Q launch.  Then the
    single-pass Algorithm 5.6 (rsvd_eigh_onepass) end to end against the two-pass route with q = 0
    (rsvd_range_finder + rsvd_eigh) on the same matrix."""
    import numpy as np
    import torch
    import paper_0909_4061_amd as rs
    from workloads import build_psd_torch

    n, k, p, q, shift = 16384, 100, 20, 1, 1e-4
    l = k + p
    dev = torch.device("cuda", 0)
    lam = 1.0 / np.arange(1, 4097, dtype=np.float64)
    exact = np.concatenate([lam + shift, np.full(n - lam.size, shift)])
    t = time.perf_counter()
    A = build_psd_torch(n, lam, shift, seed=args.seed, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    print(f"# built psd A {n}x{n} on the GPU in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream(dev)
    paths = {}
    for prec in (["bf16x3", "native"] if args.only is None else [args.only]):
        pr = rs.problem(n, n, k, p, q, dtype=A.dtype, prec=prec, seed=args.seed)
        ws = rs.Workspace(pr, dev)
        Q = rs.rsvd_range_finder(A, k, p, q=q, prec=prec, seed=args.seed, ws=ws)
        rs.rsvd_power_iter(A, Q, k, p, q, prec=prec, seed=args.seed, ws=ws)
        U = torch.empty(n, k, dtype=A.dtype, device=dev)
        Lam = torch.empty(k, dtype=A.dtype, device=dev)
        res = {}
        for name, fn in (("eigh", rs.rsvd_eigh), ("nystrom", rs.rsvd_nystrom)):
            for _ in range(args.warmup):
                fn(A, Q, k, prec=prec, U=U, Lam=Lam, ws=ws)
            torch.cuda.synchronize()
            rs.device_status(dev)
            rs.profile_enable(4 * max(args.steps, 1), dev)
            rs.profile_select(["stream_nn"], dev)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                fn(A, Q, k, prec=prec, U=U, Lam=Lam, ws=ws)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            launches, tot = rs.profile_read(dev)["stream_nn"]
            rs.profile_enable(0, dev)
            flags = rs.device_status(dev)
            err = spectral_norm_residual(A, U, Lam, U) / exact[k]
            lam_err = float(np.max(np.abs(Lam.double().cpu().numpy() - exact[:k]) / exact[:k]))
            avg_s = tot / launches / 1e3
            bytes_launch = 4.0 * n * n + 2 * 4.0 * n * l
            res[name] = {"ms_per_call": ms, "a_read_gbs": 4.0 * n * n / (ms / 1e3) / 1e9, "err_ratio": err,
                         "lambda_rel_err_vs_construction": lam_err, "flags": flags,
                         "roofline": {"bound": "hbm", "achieved": bytes_launch / avg_s / 1e9, "peak": PEAK_HBM_GBS,
                                      "unit": "GB/s", "frac": bytes_launch / avg_s / 1e9 / PEAK_HBM_GBS,
                                      "traffic": None, "kernel": f"gemm_nn_{prec}", "launches": launches,
                                      "avg_us": avg_s * 1e6, "per_launch": {"bytes": bytes_launch}}}
            print(f"# psd {prec} {name}: {ms:.3f} ms per call, err ratio {err:.4f}, "
                  f"lambda rel err {lam_err:.2e}", file=sys.stderr, flush=True)
        # Algorithm 5.6 (one pass over A) against the two-pass route it replaces (the range finder
        # with q = 0, then Algorithm 5.3): each timed end to end
        pr0 = rs.problem(n, n, k, p, 0, dtype=A.dtype, prec=prec, seed=args.seed)
        ws0 = rs.Workspace(pr0, dev)
        Q0 = torch.empty(n, l, dtype=A.dtype, device=dev)

        def two_pass():
            rs.rsvd_range_finder(A, k, p, prec=prec, seed=args.seed, Q=Q0, ws=ws0)
            rs.rsvd_eigh(A, Q0, k, prec=prec, U=U, Lam=Lam, ws=ws0)

        def one_pass():
            rs.rsvd_eigh_onepass(A, k, p, prec=prec, seed=args.seed, U=U, Lam=Lam, ws=ws0)

        for name, fn in (("onepass", one_pass), ("twopass_q0", two_pass)):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            rs.device_status(dev)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            flags = rs.device_status(dev)
            err = spectral_norm_residual(A, U, Lam, U) / exact[k]
            lam_err = float(np.max(np.abs(Lam.double().cpu().numpy() - exact[:k]) / exact[:k]))
            res[name] = {"ms_per_call": ms, "passes_over_a": 1 if name == "onepass" else 2, "err_ratio": err,
                         "lambda_rel_err_vs_construction": lam_err, "flags": flags}
            print(f"# psd {prec} {name}: {ms:.3f} ms per call, err ratio {err:.4f}, "
                  f"lambda rel err {lam_err:.2e}", file=sys.stderr, flush=True)
        paths[prec] = res
        del ws, ws0
    hp = paths[args.only or "bf16x3"]["nystrom"]
    line = {
        "metric": "psd Stage B (Algorithm 5.5 Nystrom): A read rate of one call", "value": hp["a_read_gbs"],
        "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": hp["ms_per_call"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "prec": args.only or "bf16x3", "data": "synthetic",
        "config": {"workload": f"psd eigendecomposition Stage B, FP32 {n}x{n}, lam_j = 1/j (j <= 4096) + {shift}, "
                               f"k={k}, p={p}, Q from q={q}", "n": n, "k": k, "p": p, "q": q},
        "floor_ms": 4.0 * n * n / PEAK_HBM_GBS / 1e9 * 1e3,
        "roofline": hp["roofline"], "paths": paths,
    }
    del A
    return line


def workload_batched(args):
    """512 uneven FP32 matrices, sigma_j = exp(-j/r), p = 8, q = 1, one rsvd_batched call per step."""
    import numpy as np
    import torch
    import paper_0909_4061_amd as rs
    from workloads import batch_shapes, build_matrix_torch, spectrum

    dev = torch.device("cuda", 0)
    shapes = batch_shapes(args.batch)
    p, q = 8, 1
    t = time.perf_counter()
    As, sigmas = [], []
    for i, (m, n, k, r) in enumerate(shapes):
        sig = spectrum("exp_r", min(m, n), rate=r)
        As.append(build_matrix_torch(m, n, sig, seed=args.seed + i, dtype=torch.float32, device=dev))
        sigmas.append(sig)
    torch.cuda.synchronize()
    print(f"# built {len(As)} matrices on the GPU in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    ks = [k for _, _, k, _ in shapes]
    out = {}
    for prec in (["bf16x3", "native"] if args.only is None else [args.only]):
        probs = [rs.problem(A.shape[0], A.shape[1], k, p, q, dtype=A.dtype, prec=prec, seed=args.seed,
                            stream_id=i) for i, (A, k) in enumerate(zip(As, ks))]
        ws = rs.BatchWorkspace(probs, dev)
        outs = rs.rsvd_batched(As, ks, p=p, q=q, prec=prec, seed=args.seed, ws=ws)   # records the plan
        for _ in range(args.warmup):
            rs.rsvd_batched(As, ks, p=p, q=q, prec=prec, seed=args.seed, ws=ws, outs=outs)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream(dev)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(args.steps):
            rs.rsvd_batched(As, ks, p=p, q=q, prec=prec, seed=args.seed, ws=ws, outs=outs)
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / args.steps
        flags = rs.device_status(dev)
        flops = sum(algorithmic_flops(A.shape[0], A.shape[1], k + p, k, q) for A, k in zip(As, ks))
        hbm = sum(algorithmic_bytes(A.shape[0], A.shape[1], k + p, q) for A, k in zip(As, ks))
        # accuracy: singular values against the construction, relative to
        # sigma_j + (4 sqrt(m) + 2 l) u_32 sigma_1 (below that level FP32
        # arithmetic resolves nothing); residual ratio on a sample of 16
        rel = []
        for (U, S, V), sig, k, A in zip(outs, sigmas, ks, As):
            s_ = S.double().cpu().numpy()
            floor = (4.0 * np.sqrt(max(A.shape)) + 2.0 * (k + p)) * 2.0 ** -24 * sig[0]
            rel.append(float(np.max(np.abs(s_ - sig[:k]) / (sig[:k] + floor))))
        ratios = []
        for i in np.linspace(0, len(As) - 1, 16).astype(int):
            U, S, V = outs[i]
            k = ks[i]
            if k < len(sigmas[i]):
                ratios.append(spectral_norm_residual(As[i], U, S, V) / sigmas[i][k])
        out[prec] = {"ms_per_step": ms, "tflops": flops / (ms / 1e3) / 1e12, "hbm_gbs": hbm / (ms / 1e3) / 1e9,
                     "sigma_rel_err_max": max(rel), "err_ratio_median": float(np.median(ratios)),
                     "err_ratio_max": float(np.max(ratios)), "flags": flags}
        print(f"# {prec}: {ms:.3f} ms/batch, {out[prec]['tflops']:.2f} TFLOP/s, err ratio median "
              f"{out[prec]['err_ratio_median']:.3f}", file=sys.stderr, flush=True)
    head = "bf16x3" if "bf16x3" in out else "native"
    hp = out[head]
    line = {
        "metric": "rSVD TFLOP/s + HBM GB/s at stated ||A-USV*||/sigma_{k+1}; BF16-MFMA vs FP32",
        "value": hp["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": hp["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if head == "bf16x3" else "f32", "prec": head, "data": "synthetic",
        "config": {"workload": f"batched rSVD, {len(As)} uneven FP32 matrices (m<=2048, n<=1024), "
                               f"sigma_j=exp(-j/r), p={p}, q={q}, one graph-replayed rsvd_batched call per step",
                   "count": len(As), "p": p, "q": q, "sketch": "gaussian"},
        "hbm_gbs": hp["hbm_gbs"], "err_ratio": hp["err_ratio_median"], "paths": out,
    }
    return line


def workload_differentiable(args):
    """32 FP32 4096 x 2048 matrices, sigma_j = j^-1/2, k = 64, p = 16, q = 1: forward, the loss
    ||U S V^T - T||_F^2 + w . S and its gradient in A through the hand-written adjoint."""
    import numpy as np
    import torch
    import paper_0909_4061_amd as rs
    from workloads import CONFIGS, build_matrix_torch, spectrum

    cfg = CONFIGS["differentiable_32x4096x2048"]
    m, n, k, p, q, count = cfg.m, cfg.n, cfg.k, cfg.p, cfg.q, args.batch_diff
    l = k + p
    dev = torch.device("cuda", 0)
    sig = spectrum(cfg.spectrum, min(m, n))
    t = time.perf_counter()
    As, Ts, ws_ = [], [], []
    for i in range(count):
        As.append(build_matrix_torch(m, n, sig, seed=args.seed + i, dtype=torch.float32, device=dev))
        gen = torch.Generator(device=dev)
        gen.manual_seed(args.seed + 1000 + i)
        Ts.append(torch.randn(m, n, generator=gen, device=dev, dtype=torch.float32))
        ws_.append(torch.rand(k, generator=gen, device=dev, dtype=torch.float32))
    torch.cuda.synchronize()
    print(f"# built {count} matrices on the GPU in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    prec = args.only or "bf16x3"

    # batched (default): one rsvd_batched call for all matrices, one stacked loss, and one
    # rsvd_backward_batched call from autograd -- every step of the forward and of the adjoint is one
    # launch over all matrices, replayed from a graph.
    # streams: matrix i runs (forward, loss, adjoint) alone on stream i mod S, so the latency-bound
    # small steps of different matrices overlap (autograd runs each backward op on the stream of its
    # forward op; workspaces come from the allocator of the current stream).
    nstreams = max(1, args.diff_streams)
    streams = [torch.cuda.Stream(device=dev) for _ in range(nstreams)] if args.diff_mode == "streams" else []
    T3 = torch.stack(Ts) if args.diff_mode == "batched" else None
    W3 = torch.stack(ws_) if args.diff_mode == "batched" else None
    if T3 is not None:
        del Ts[:]

    # ||U S V^T - T||_F^2 = tr(U^T U S V^T V S) - 2 sum_j s_j u_j^T T v_j + ||T||_F^2 for any U, V:
    # the same loss (and the same gradients in U, S, V) from one (m x n)(n x k) product per
    # matrix instead of the m x n residual.
    T3sq = T3.square().sum() if T3 is not None else None

    def step_batched():
        leaves = [A.detach().requires_grad_(True) for A in As]
        outs = rs.rsvd_batched(leaves, k, p=p, q=q, seed=args.seed, prec=prec, keep_state=args.keep_state)
        U3 = torch.stack([o[0] for o in outs])
        S3 = torch.stack([o[1] for o in outs])
        V3 = torch.stack([o[2] for o in outs])
        TV = torch.bmm(T3, V3)  # m x k per matrix
        GU = torch.bmm(U3.transpose(1, 2).contiguous(), U3)
        GV = torch.bmm(V3.transpose(1, 2).contiguous(), V3)
        quad = (GU * GV * (S3[:, :, None] * S3[:, None, :])).sum()
        cross = (S3 * (U3 * TV).sum(dim=1)).sum()
        L = quad - 2.0 * cross + T3sq + (W3 * S3).sum()
        L.backward()
        return [x.grad for x in leaves]

    def step():
        if args.diff_mode == "batched":
            return step_batched()
        cur = torch.cuda.current_stream(dev)
        for s_ in streams:
            s_.wait_stream(cur)
        grads = []
        for i in range(count):
            with torch.cuda.stream(streams[i % nstreams]):
                A = As[i].detach().requires_grad_(True)
                U, S, V = rs.rsvd(A, k, p, q, seed=args.seed, stream_id=i, prec=prec, keep_state=args.keep_state)
                L = ((U * S[None, :]) @ V.T - Ts[i]).square().sum() + (ws_[i] * S).sum()
                L.backward()
                grads.append(A.grad)
        for s_ in streams:
            cur.wait_stream(s_)
        return grads

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(args.steps):
        grads = step()
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    fwd = algorithmic_flops(m, n, l, k, q)
    # adjoint: (2q + 1) products with A in reverse and gA = Left RightT with K = (2q + 2) l (the
    # recomputation of the forward that the default adjoint makes is not counted)
    bwd = (2 * q + 1) * 2.0 * m * n * l + 2.0 * m * n * (2 * q + 2) * l
    flops = count * (fwd + bwd)
    # loss-side products in torch (U S V^T - T and its derivatives) are not counted
    hbm = count * (algorithmic_bytes(m, n, l, q) + (2 * q + 1) * m * n * 4 + m * n * 4)
    gnorm = float(torch.stack([g.norm() for g in grads]).mean())
    line = {
        "metric": "rSVD TFLOP/s + HBM GB/s at stated ||A-USV*||/sigma_{k+1}; BF16-MFMA vs FP32",
        "value": flops / (ms / 1e3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16" if prec == "bf16x3" else "f32", "prec": prec, "data": "synthetic",
        "config": {"workload": f"differentiable rSVD, {count} x FP32 {m}x{n}, sigma_j=j^-1/2, k={k}, p={p}, q={q}, "
                               "forward + loss + hand-written adjoint per matrix",
                   "count": count, "m": m, "n": n, "k": k, "p": p, "q": q, "mode": args.diff_mode,
                   "adjoint": "kept forward state" if args.keep_state else "forward recomputed",
                   **({"streams": nstreams} if args.diff_mode == "streams" else {})},
        "hbm_gbs": hbm / (ms / 1e3) / 1e9, "ms_per_matrix": ms / count, "mean_grad_norm": gnorm,
    }
    return line


def measured_traffic(family, prec, m, n, l):
    """Counter-measured HBM bytes per launch, or None if the kernel source or shape differs."""
    import hashlib
    src = os.path.join(ROOT, "paper_0909_4061_amd", "csrc", "k_stream.hip")
    try:
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if sha != TRAFFIC_KERNEL_SHA or (m, n, l) != TRAFFIC_SHAPE:
        return None
    return TRAFFIC_BYTES.get(f"{family}_{prec}")


def roofline_for(res, m, n, l, prec):
    """Roofline figures of the dominant kernel (the GEMM family that streams A
    and takes the most time), from the live per-launch event timing."""
    fam = max(("stream_nn", "stream_tn"), key=lambda f: res["prof"][f][1])
    launches, total_ms = res["prof"][fam]
    avg_s = total_ms / launches / 1e3
    rows, K = (m, n) if fam == "stream_nn" else (n, m)
    bytes_launch = 4.0 * (rows * K + (rows + K) * l)
    flops_launch = 2.0 * rows * K * l
    if prec == "native":
        achieved = flops_launch / avg_s / 1e12
        out = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
               "frac": achieved / PEAK_TFLOPS["f32"]}
    else:
        achieved = bytes_launch / avg_s / 1e9
        out = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
               "frac": achieved / PEAK_HBM_GBS}
    out.update({"kernel": f"gemm_{'tn' if fam == 'stream_tn' else 'nn'}_{'f32' if prec == 'native' else prec}",
                "launches": launches, "avg_us": avg_s * 1e6, "traffic": measured_traffic(fam, prec, m, n, l),
                "per_launch": {"bytes": bytes_launch, "flops": flops_launch}})
    return out


def workload_fp64(args):
    """FP64 2000 x 1000, sigma_j = exp(-j/20), k = 20, p = 10, q = 0: a latency-scale problem (its
    A is 16 MB).  Reports microseconds per rSVD next to the HBM and FP64-MFMA floors."""
    import torch
    from workloads import CONFIGS, build_matrix_torch, spectrum

    cfg = CONFIGS["fp64_2000x1000"]
    m, n, k, p, q = cfg.m, cfg.n, cfg.k, cfg.p, cfg.q
    l = k + p
    dev = torch.device("cuda", 0)
    sigma = spectrum(cfg.spectrum, min(m, n))
    A = build_matrix_torch(m, n, sigma, seed=args.seed, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    steps = args.steps if args.steps is not None else 200
    warmup = args.warmup
    res = run_path(A, k, p, q, "native", steps, warmup, args.seed)
    err = spectral_norm_residual(A, res["U"], res["S"], res["V"]) / sigma[k]
    # the same rSVD through rsvd_full: the four calls' launches captured once in a HIP graph and
    # replayed (no host work per kernel)
    import paper_0909_4061_amd as rs
    pr = rs.problem(m, n, k, p, q, dtype=A.dtype, seed=args.seed)
    fws = rs.full_workspace(pr, dev)
    outs = rs.rsvd_full(A, k, p, q, seed=args.seed, ws=fws)
    for _ in range(warmup):
        rs.rsvd_full(A, k, p, q, seed=args.seed, outs=outs, ws=fws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        rs.rsvd_full(A, k, p, q, seed=args.seed, outs=outs, ws=fws)
    e1.record()
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / steps
    graph_err = spectral_norm_residual(A, *outs) / sigma[k]
    flops = algorithmic_flops(m, n, l, k, q)
    nbytes = algorithmic_bytes(m, n, l, q, esize=8)
    s = res["ms_per_step"] / 1e3
    floor_hbm_us = nbytes / (PEAK_HBM_GBS * 1e9) * 1e6
    floor_mfma_us = flops / (PEAK_TFLOPS["f64"] * 1e12) * 1e6
    achieved = nbytes / s / 1e9
    line = {
        "metric": "rSVD TFLOP/s + HBM GB/s at stated ||A-USV*||/sigma_{k+1}; BF16-MFMA vs FP32",
        "value": flops / s / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": res["ms_per_step"], "us_per_rsvd": res["ms_per_step"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "prec": "native", "data": "synthetic",
        "config": {"workload": f"FP64 rSVD {m}x{n}, sigma_j=exp(-j/20), k={k}, p={p}, q={q}",
                   "m": m, "n": n, "k": k, "p": p, "q": q},
        "hbm_gbs": achieved, "err_ratio": err, "flags": res["flags"],
        # the whole step against its floors: at this size every kernel is a few
        # microseconds and the step is bound by the chain of dependent launches
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None, "scope": "whole step",
                     "floor_us": {"hbm": floor_hbm_us, "mfma_f64": floor_mfma_us}},
        "kernel_ms_per_step": res["breakdown"],
        "graph_replay": {"entry": "rsvd_full", "ms_per_step": graph_ms,
                         "us_per_rsvd": graph_ms * 1e3, "tflops": flops / (graph_ms / 1e3) / 1e12,
                         "err_ratio": graph_err},
    }
    return line


def measured_ceilings(A, reps=10):
    """Achievable peaks on this GPU from the library's probe kernels (measurement aids, not part of
    the method): a streaming read of A with 16-byte loads, and MFMA loops in BF16, FP32 and FP64."""
    import torch
    import paper_0909_4061_amd as rs
    dev = A.device
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    out = {}
    nbytes = rs.probe_hbm_read(A)[1]
    out["hbm_read_gbs"] = nbytes / timed(lambda: rs.probe_hbm_read(A)) / 1e9
    blocks = 4 * MI355X_CUS
    for kind, iters in (("bf16", 4096), ("fp32", 4096), ("fp64", 2048)):
        flops = rs.probe_mfma(kind, iters, blocks, dev)[1]
        out[f"mfma_{kind}_tflops"] = flops / timed(lambda: rs.probe_mfma(kind, iters, blocks, dev)) / 1e12
    out["how"] = (f"library probe kernels: one streaming read of the {nbytes}-byte input (16-byte loads, "
                  f"2048 workgroups); MFMA loops of four independent accumulations per wave, {blocks} "
                  f"workgroups of four waves; {reps} repetitions each")
    return out


def cpu_baseline(A, k, p, q, seed, flops, budget_s=30.0, paths_out=None, sigma=None):
    """The FP64 oracle on the host cores, on a bounded sample of the workload.

    The sample is the first m' rows of A with m' chosen so that one run takes
    about budget_s (at most all m rows); the rate is scaled to the same
    algorithmic-flop unit as the GPU line.  When the sample is the whole matrix
    (or after one more oracle run on it), the GPU paths' results are compared
    with the oracle's: the largest relative singular-value difference over the
    k retained values, and the ratio of residual norms ||A - U S V*||_2 (the
    benchmark's evaluator applied to both factorizations)."""
    import numpy as np
    import torch
    from oracle import rsvd as orsvd
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 0) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threads = os.cpu_count()
    m, n = A.shape
    # calibrate on a small slab, then size the sample
    mc = min(m, 2048)
    A_c = A[:mc].double().cpu().numpy()
    t = time.perf_counter()
    orsvd.rsvd(A_c, k, p, q, seed=seed, dtype=np.float32)
    tc = time.perf_counter() - t
    mm = int(min(m, max(mc, mc * budget_s / max(tc, 1e-3))))
    mm = max(mm, k + p)
    A_s = A[:mm].double().cpu().numpy()
    t = time.perf_counter()
    ref = orsvd.rsvd(A_s, k, p, q, seed=seed, dtype=np.float32)
    dt = time.perf_counter() - t
    f_s = algorithmic_flops(mm, n, k + p, k, q)
    out = {"value": f_s / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
           "sample": f"FP64 numpy oracle, full rSVD (k={k}, p={p}, q={q}) on the first {mm} of {m} rows "
                     f"of the same matrix, {dt:.1f} s",
           "seconds": dt, "rows": mm}
    if paths_out:
        if mm < m:
            ref = orsvd.rsvd(A.double().cpu().numpy(), k, p, q, seed=seed, dtype=np.float32)
        Uo, So, Vo = (torch.from_numpy(ref[x]).to(A.device) for x in ("Uk", "Sk", "Vk"))
        res_o = spectral_norm_residual(A, Uo, So, Vo)
        parity = {"oracle_err_ratio": res_o / sigma[k] if sigma is not None else None}
        for name, (U, S, V) in paths_out.items():
            Sg = S.double().cpu().numpy()
            parity[name] = {"sigma_rel_err_max": float(np.max(np.abs(Sg - ref["Sk"]) / ref["Sk"])),
                            "res_ratio": spectral_norm_residual(A, U, S, V) / res_o}
        out["parity_vs_oracle"] = parity
    return out


def compact_sub_workloads(args):
    """The other workloads, timed briefly (args.sub_steps steps each) so that the default run covers
    them; each full line is available with --workload."""
    import copy
    import numpy as np
    import torch
    from workloads import build_matrix_torch, spectrum
    out = {}
    sub = copy.copy(args)
    sub.steps, sub.warmup, sub.only = args.sub_steps, 2, None

    def guarded(name, fn):
        t = time.perf_counter()
        try:
            out[name] = fn()
        except Exception as e:  # a failing sub-workload is reported, not fatal to the headline line
            out[name] = {"error": f"{type(e).__name__}: {e}"}
        out[name]["wall_s"] = time.perf_counter() - t
        torch.cuda.empty_cache()
        print(f"# {name}: {json.dumps(out[name])[:300]}", file=sys.stderr, flush=True)

    def fp64():
        f = copy.copy(sub)
        f.steps = 200
        d = workload_fp64(f)
        return {"us_per_rsvd": d["us_per_rsvd"], "graph_us_per_rsvd": d["graph_replay"]["us_per_rsvd"],
                "err_ratio": d["err_ratio"], "floor_us": d["roofline"]["floor_us"], "steps": f.steps}

    def srft():
        m, n, k, p = 32768, 16384, 50, 78
        sigma = spectrum("gap", n)
        A = build_matrix_torch(m, n, sigma, seed=args.seed, dtype=torch.float32, device=torch.device("cuda", 0))
        s2 = copy.copy(sub)
        s2.k, s2.p = k, p
        d = workload_srft(s2, A, sigma)
        del A
        return {"srft": {x: d["paths"]["srft"][x] for x in ("ms_per_step", "stage_a_ms", "err_ratio", "tflops")},
                "gaussian": {x: d["paths"]["gaussian"][x] for x in ("ms_per_step", "stage_a_ms", "err_ratio",
                                                                    "tflops")},
                "gsrft": {x: d["paths"]["gsrft"][x] for x in ("ms_per_step", "stage_a_ms", "err_ratio", "tflops")},
                "stage_a_speedup_vs_gaussian": d["stage_a_speedup_vs_gaussian"],
                "roofline_srft_kernel": {x: d["roofline"][x] for x in ("achieved", "frac", "avg_us")},
                "roofline_gsrft_pretransform": {x: d["gsrft_pretransform"][x] for x in ("achieved", "frac", "avg_us")},
                "steps": s2.steps}

    def batched():
        s2 = copy.copy(sub)
        s2.only = "bf16x3"
        d = workload_batched(s2)
        pth = d["paths"]["bf16x3"]
        return {x: pth[x] for x in ("ms_per_step", "tflops", "err_ratio_median", "err_ratio_max",
                                    "sigma_rel_err_max")} | {"count": d["config"]["count"], "steps": s2.steps}

    def differentiable():
        d = workload_differentiable(sub)
        return {x: d[x] for x in ("ms_per_step", "value", "ms_per_matrix")} | {
            "unit": d["unit"], "adjoint": d["config"]["adjoint"], "count": d["config"]["count"],
            "steps": sub.steps}

    guarded("fp64_2000x1000", fp64)
    guarded("srft_32768x16384", srft)
    guarded("batched_512", batched)
    def psd():
        s2 = copy.copy(sub)
        s2.only = "bf16x3"
        d = workload_psd(s2)
        pth = d["paths"]["bf16x3"]
        out_ = {name: {x: pth[name][x] for x in ("ms_per_call", "a_read_gbs", "err_ratio",
                                                 "lambda_rel_err_vs_construction")}
                | {"stream_nn_frac": pth[name]["roofline"]["frac"]} for name in ("eigh", "nystrom")}
        out_ |= {name: {x: pth[name][x] for x in ("ms_per_call", "err_ratio", "passes_over_a")}
                 for name in ("onepass", "twopass_q0")}
        return out_ | {"floor_ms": d["floor_ms"], "steps": s2.steps}

    guarded("differentiable_32x4096x2048", differentiable)
    guarded("psd_stage_b_16384", psd)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 10; 200 for the fp64 workload)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--m", type=int, default=16384)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--p", type=int, default=20)
    ap.add_argument("--q", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0x09094061)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sub", action="store_true", help="skip the brief runs of the other workloads")
    ap.add_argument("--sub-steps", type=int, default=5, help="timed steps of each other workload in the default run")
    ap.add_argument("--only", choices=["bf16x3", "native"], default=None)
    ap.add_argument("--input", choices=["construct", "randn"], default="construct",
                    help="construct: A = U diag(1/j) V^T (the workload); randn: i.i.d. Gaussian A of the "
                         "same shape, for hardware-counter runs only (byte counts do not depend on values)")
    ap.add_argument("--batch", type=int, default=512, help="matrices in the batched workload")
    ap.add_argument("--diff-mode", choices=("batched", "streams"), default="batched",
                    help="differentiable workload: one batched forward and adjoint, or one call per matrix "
                         "over concurrent streams")
    ap.add_argument("--diff-streams", type=int, default=8,
                    help="streams the differentiable workload's independent matrices are spread over")
    ap.add_argument("--batch-diff", type=int, default=32, help="matrices in the differentiable workload")
    ap.add_argument("--keep-state", action="store_true",
                    help="differentiable workload: the forward keeps its bases for the adjoint instead of the "
                         "adjoint recomputing them")
    ap.add_argument("--workload", choices=["power", "srft", "batched", "differentiable", "fp64", "psd", "onepass"],
                    default="power",
                    help="power: the power-iteration rSVD (default); srft: SRFT vs Gaussian sketch, "
                         "FP32 32768 x 16384 with a spectral gap, k = 50, p = 78, q = 0; batched: 512 "
                         "uneven FP32 matrices, p = 8, q = 1; differentiable: 32 FP32 4096 x 2048 "
                         "matrices, forward + loss + adjoint; fp64: FP64 2000 x 1000, k = 20, p = 10, "
                         "q = 0 (200 steps unless --steps is given); psd: Stage B for a 16384 x 16384 "
                         "psd matrix (Algorithms 5.3 and 5.5), k = 100, p = 20; onepass: the two-sided "
                         "single pass (Section 5.5) against the two-pass route with q = 0 on the power "
                         "workload's matrix")
    ap.add_argument("--srft-prec", choices=["bf16x3", "native"], default="bf16x3",
                    help="arithmetic of the GEMMs that stream A in the srft workload")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain device copy of A (known size) before the paths, to scale "
                         "HBM byte counters in profiling runs")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from workloads import build_matrix_torch, spectrum

    if args.workload == "fp64":
        print(json.dumps(workload_fp64(args)))
        return
    if args.steps is None:
        args.steps = 10
    if args.workload == "batched":
        print(json.dumps(workload_batched(args)))
        return
    if args.workload == "differentiable":
        print(json.dumps(workload_differentiable(args)))
        return
    if args.workload == "psd":
        print(json.dumps(workload_psd(args)))
        return
    if args.workload == "srft":
        args.m, args.n, args.k, args.p, args.q = 32768, 16384, 50, 78, 0
    m, n, k, p, q = args.m, args.n, args.k, args.p, args.q
    l = k + p
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t = time.perf_counter()
    sigma = spectrum("inv" if args.workload in ("power", "onepass") else "gap", min(m, n))
    if args.input == "construct":
        A = build_matrix_torch(m, n, sigma, seed=args.seed, dtype=torch.float32, device=dev)
    else:
        gen = torch.Generator(device=dev)
        gen.manual_seed(args.seed)
        A = torch.randn(m, n, generator=gen, device=dev, dtype=torch.float32)
    torch.cuda.synchronize()
    print(f"# built A {m}x{n} on the GPU in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)

    if args.calib_copy:
        Ac = A.clone()
        torch.cuda.synchronize()
        print(f"# calibration copy: {A.numel() * A.element_size()} bytes read and written",
              file=sys.stderr, flush=True)
        del Ac

    if args.workload == "srft":
        print(json.dumps(workload_srft(args, A, sigma)))
        return
    if args.workload == "onepass":
        prec = args.only or "bf16x3"
        res = single_pass_general(A, k, p, sigma, prec, args.steps, args.warmup, args.seed)
        one = res["onepass"]
        print(json.dumps({
            "metric": "two-sided single pass (Section 5.5): time per factorization", "value": one["ms_per_call"],
            "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": one["ms_per_call"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16" if prec == "bf16x3" else "f32", "prec": prec, "data": "synthetic",
            "config": {"workload": f"two-sided single pass, FP32 {m}x{n}, sigma_j=1/j, k={k}, p={p}",
                       "m": m, "n": n, "k": k, "p": p},
            "paths": res}))
        return

    flops = algorithmic_flops(m, n, l, k, q)
    hbm = algorithmic_bytes(m, n, l, q)
    paths, factors = {}, {}
    for prec in (["bf16x3", "native"] if args.only is None else [args.only]):
        res = run_path(A, k, p, q, prec, args.steps, args.warmup, args.seed)
        err = spectral_norm_residual(A, res["U"], res["S"], res["V"]) / sigma[k]
        sig_err = float(np.max(np.abs(res["S"].double().cpu().numpy() - sigma[:k]) / sigma[:k]))
        s = res["ms_per_step"] / 1e3
        fl = e2e_floor(m, n, l, k, q, prec)
        paths[prec] = {
            "ms_per_step": res["ms_per_step"], "tflops": flops / s / 1e12, "hbm_gbs": hbm / s / 1e9,
            "err_ratio": err, "sigma_rel_err_vs_construction": sig_err, "flags": res["flags"],
            "e2e_roofline": fl | {"frac": fl["floor_ms"] / res["ms_per_step"]},
            "roofline": roofline_for(res, m, n, l, prec),
            "kernel_ms_per_step": res["breakdown"],
        }
        factors[prec] = (res["U"].clone(), res["S"].clone(), res["V"].clone())
        print(f"# {prec}: {res['ms_per_step']:.3f} ms/step, {paths[prec]['tflops']:.2f} TFLOP/s, "
              f"err ratio {err:.4f}, {paths[prec]['e2e_roofline']['frac']:.3f} of the step's floor",
              file=sys.stderr, flush=True)

    head = "bf16x3" if "bf16x3" in paths else "native"
    hp = paths[head]
    line = {
        "metric": "rSVD TFLOP/s + HBM GB/s at stated ||A-USV*||/sigma_{k+1}; BF16-MFMA vs FP32",
        "value": hp["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": hp["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if head == "bf16x3" else "f32", "prec": head, "data": "synthetic",
        "config": {"workload": f"power-iteration rSVD, FP32 {m}x{n}, sigma_j=1/j, k={k}, p={p}, q={q}"
                               + ("" if args.input == "construct" else " (Gaussian input: counter run)"),
                   "m": m, "n": n, "k": k, "p": p, "q": q, "sketch": "gaussian"},
        "hbm_gbs": hp["hbm_gbs"], "err_ratio": hp["err_ratio"], "roofline": hp["roofline"],
        "e2e_roofline": hp["e2e_roofline"],
        "paths": paths,
    }
    if "native" in paths and head != "native":
        line["speedup_vs_fp32"] = paths["native"]["ms_per_step"] / hp["ms_per_step"]
    if args.input == "construct":
        line["single_pass_two_sided"] = single_pass_general(A, k, p, sigma, head, args.steps, args.warmup,
                                                            args.seed)
    ceil = measured_ceilings(A)
    line["measured_ceilings"] = ceil
    for d in [line["roofline"]] + [pd["roofline"] for pd in line["paths"].values()]:
        d["frac_of_measured"] = d["achieved"] / (ceil["hbm_read_gbs"] if d["bound"] == "hbm"
                                                 else ceil["mfma_fp32_tflops"])
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(A, k, p, q, args.seed, flops, paths_out=factors, sigma=sigma)
        print(f"# parity vs oracle: {json.dumps(line['cpu_baseline'].get('parity_vs_oracle'))}", file=sys.stderr,
              flush=True)
    del A, factors
    torch.cuda.empty_cache()
    if not args.no_sub:
        line["workloads"] = compact_sub_workloads(args)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
