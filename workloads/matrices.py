"""Seeded test matrices A = U diag(sigma) V^T and the benchmark configurations.

Random numbers here come from numpy's Philox bit generator (CPU) or torch's
generator (GPU builds of the large matrices); they are input data, not the
method's own draws.  Streams: 1 = U, 2 = V, 3 = random parts of a spectrum,
4 = batch shapes, 5 = regression targets, 6 = loss weights.
"""

import math
from dataclasses import dataclass, field

import numpy as np

SEED = 0x09094061

STREAM_U, STREAM_V, STREAM_SIGMA, STREAM_SHAPES, STREAM_T, STREAM_W = 1, 2, 3, 4, 5, 6


def _rng(seed, stream):
    return np.random.Generator(np.random.Philox(key=np.array([seed, stream], dtype=np.uint64)))


@dataclass(frozen=True)
class Config:
    """One workload: sizes, rSVD parameters and the spectrum recipe."""
    name: str
    m: int
    n: int
    k: int
    p: int
    q: int
    dtype: str              # "f64" or "f32": the storage type of A
    spectrum: str           # "exp20", "inv", "gap", "exp_r", "invsqrt"
    sketch: str = "gaussian"
    batch: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def l(self):
        return self.k + self.p


CONFIGS = {
    # Plain rSVD in FP64: sigma_j = exp(-j/20), Gaussian Omega 1000 x 30.
    "fp64_2000x1000": Config("fp64_2000x1000", 2000, 1000, 20, 10, 0, "f64", "exp20"),
    # Power-iteration rSVD, FP32 16384 x 8192, sigma_j = 1/j, q = 2.
    "power_16384x8192": Config("power_16384x8192", 16384, 8192, 100, 20, 2, "f32", "inv"),
    # SRFT vs Gaussian sketch, FP32 32768 x 16384 with a spectral gap, l = 128.
    "srft_32768x16384": Config("srft_32768x16384", 32768, 16384, 50, 78, 0, "f32", "gap", sketch="srft"),
    # 512 uneven FP32 matrices, p = 8, q = 1 (shapes from batch_shapes()).
    "batched_512": Config("batched_512", 2048, 1024, 64, 8, 1, "f32", "exp_r", batch=512),
    # Differentiable rSVD: 32 x (4096 x 2048), sigma_j = j^-1/2, k = 64, p = 16, q = 1.
    "differentiable_32x4096x2048": Config("differentiable_32x4096x2048", 4096, 2048, 64, 16, 1, "f32", "invsqrt", batch=32),
}


def spectrum(kind, r, seed=SEED, rate=None):
    """The r singular values sigma_1 >= ... >= sigma_r of a recipe, FP64.

    exp20    sigma_j = exp(-j/20)
    exp_r    sigma_j = exp(-j/rate)
    inv      sigma_j = 1/j
    invsqrt  sigma_j = j^(-1/2)
    gap      sigma_1..50 uniform in [1, 2] (sorted descending), then
             sigma_j = |1e-3 (1 + 0.1 g_j)| with g_j standard normal, sorted
    """
    j = np.arange(1, r + 1, dtype=np.float64)
    if kind == "exp20":
        return np.exp(-j / 20.0)
    if kind == "exp_r":
        return np.exp(-j / float(rate))
    if kind == "inv":
        return 1.0 / j
    if kind == "invsqrt":
        return j ** -0.5
    if kind == "gap":
        g = _rng(seed, STREAM_SIGMA)
        head = np.sort(g.uniform(1.0, 2.0, size=min(50, r)))[::-1]
        tail = np.sort(np.abs(1e-3 * (1.0 + 0.1 * g.standard_normal(max(r - 50, 0)))))[::-1]
        return np.concatenate([head, tail])
    raise ValueError(f"unknown spectrum {kind!r}")


def haar_factor(rows, cols, seed, stream):
    """Q factor (diag(R) > 0) of a seeded rows x cols standard Gaussian matrix."""
    G = _rng(seed, stream).standard_normal((rows, cols))
    Q, R = np.linalg.qr(G, mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def build_matrix(m, n, sigma, seed=SEED, dtype=np.float64, return_factors=False):
    """A = U diag(sigma) V^T in FP64, then rounded to `dtype`, on the CPU.

    U is m x r and V is n x r with r = min(m, n) = len(sigma).
    """
    r = min(m, n)
    sigma = np.asarray(sigma, dtype=np.float64)
    assert sigma.shape == (r,)
    U = haar_factor(m, r, seed, STREAM_U)
    V = haar_factor(n, r, seed, STREAM_V)
    A = (U * sigma[None, :]) @ V.T
    A = A.astype(dtype)
    if return_factors:
        return A, U, V
    return A


def build_matrix_torch(m, n, sigma, seed=SEED, dtype=None, device="cuda"):
    """Same recipe as build_matrix, built on a GPU with torch (for the large configs).

    The Gaussian draws come from torch's generator, so the matrix differs from
    build_matrix's for the same seed; every comparison against the oracle feeds
    the oracle the exact array the GPU path read.  Returns a torch tensor.
    """
    import torch

    r = min(m, n)
    dtype = dtype or torch.float32
    gen = torch.Generator(device=device)
    sig = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)

    def factor(rows, stream):
        gen.manual_seed((seed * 1000003 + stream) & 0x7FFFFFFFFFFFFFFF)
        G = torch.randn(rows, r, generator=gen, device=device, dtype=torch.float64)
        Q, R = torch.linalg.qr(G, mode="reduced")
        del G
        s = torch.sign(torch.diagonal(R))
        s[s == 0] = 1.0
        return Q * s[None, :]

    U = factor(m, STREAM_U)
    U.mul_(sig[None, :])
    V = factor(n, STREAM_V)
    A = torch.matmul(U, V.T)
    del U, V
    out = A.to(dtype)
    del A
    return out


def batch_shapes(count=512, p=8, seed=SEED):
    """Shapes, ranks and decay rates of the uneven batch.

    m log-uniform in [64, 2048], n log-uniform in [64, 1024] with n <= m (by
    rejection), rate r uniform in [2, 32], k uniform integer in [4, 64] clamped
    to k <= n - p so that l = k + p <= min(m, n).
    """
    g = _rng(seed, STREAM_SHAPES)
    out = []
    while len(out) < count:
        m = int(round(math.exp(g.uniform(math.log(64), math.log(2048)))))
        n = int(round(math.exp(g.uniform(math.log(64), math.log(1024)))))
        r = float(g.uniform(2.0, 32.0))
        k = int(g.integers(4, 65))
        if n > m:
            continue
        k = min(k, n - p)
        out.append((m, n, k, r))
    return out


def grad_targets(m, n, k, seed=SEED, index=0):
    """Regression target T (m x n, standard normal) and weights w (k, uniform [0, 1])."""
    gT = _rng(seed + index, STREAM_T)
    gW = _rng(seed + index, STREAM_W)
    return gT.standard_normal((m, n)), gW.uniform(0.0, 1.0, size=k)


STREAM_SYM = 7


def build_symmetric(n, lam, seed=SEED, dtype=np.float64, return_factors=False):
    """A = V diag(lam) V^T (n x n, symmetric) in FP64, then rounded to `dtype`, on the CPU.

    V (n x r, r = len(lam) <= n) is the Q factor (diag(R) > 0) of a seeded standard
    Gaussian matrix, so the nonzero eigenvalues of A are exactly lam in exact
    arithmetic (any signs; all lam >= 0 gives a positive semidefinite A).  The
    FP64 product is replaced by its symmetric part before rounding, so A is
    exactly symmetric in `dtype`.
    """
    lam = np.asarray(lam, dtype=np.float64)
    V = haar_factor(n, lam.size, seed, STREAM_SYM)
    A = (V * lam[None, :]) @ V.T
    A = (0.5 * (A + A.T)).astype(dtype)
    if return_factors:
        return A, V
    return A


def build_psd_torch(n, lam, shift, seed=SEED, dtype=None, device="cuda"):
    """A = V diag(lam) V^T + shift I (n x n, positive semidefinite for lam, shift >= 0) on a GPU.

    For the large configurations: V is n x r with r = len(lam) (a thin Q factor of
    a seeded Gaussian matrix from torch's generator, diag(R) > 0), so the
    eigenvalues are lam + shift (r of them) and shift (the other n - r).  Built
    in FP64, symmetrized, rounded to `dtype`.  Returns a torch tensor.
    """
    import torch

    dtype = dtype or torch.float32
    lam_t = torch.as_tensor(np.asarray(lam, dtype=np.float64), device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed((seed * 1000003 + STREAM_SYM) & 0x7FFFFFFFFFFFFFFF)
    G = torch.randn(n, lam_t.numel(), generator=gen, device=device, dtype=torch.float64)
    V, R = torch.linalg.qr(G, mode="reduced")
    del G
    s = torch.sign(torch.diagonal(R))
    s[s == 0] = 1.0
    V = V * s[None, :]
    A = torch.matmul(V * lam_t[None, :], V.T)
    del V
    A.diagonal().add_(shift)
    A = 0.5 * (A + A.T)
    out = A.to(dtype)
    del A
    return out
