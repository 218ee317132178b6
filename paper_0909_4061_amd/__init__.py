"""Randomized SVD (Halko, Martinsson, Tropp) on MI355X: Python binding of librsvd.so.

The binding only marshals arguments: torch tensors supply device pointers and
the current HIP stream, and every step of the method runs in the library's
HIP kernels.  The C entry points (include/rsvd.h) appear here under the same
names:

    rsvd_range_finder(A, k, p, ...)      -> Q       Stage A, first application
    rsvd_power_iter(A, Q, k, p, q, ...)  -> Q       Stage A, q power steps (in place)
    rsvd_project(A, Q, k, p, ...)        -> Bt      Stage B step 1 (Bt = B^T, n x l)
    rsvd_svd(Bt, Q, k, p, ...)           -> U, S, V Stage B steps 2-3 + truncation
    rsvd_eigh(A, Q, k, ...)              -> U, Lam  Stage B for symmetric A (Algorithm 5.3)
    rsvd_nystrom(A, Q, k, ...)           -> U, Lam  Stage B for psd A (Algorithm 5.5)
    rsvd_eigh_onepass(A, k, p, ...)      -> U, Lam  one pass over symmetric A (Algorithm 5.6)
    rsvd_svd_onepass(A, k, p, ...)       -> U, S, V single-pass factorization of a general A

and rsvd(A, k, p, q, ...) runs the first four.  If the library is missing the import
of any of these raises; there is no other implementation.
"""

import ctypes

import torch

from . import _lib
from ._lib import (  # noqa: F401
    RSVD_BF16, RSVD_BF16X3, RSVD_F32, RSVD_F64, RSVD_FLAG_NOCONV, RSVD_FLAG_NONFINITE,
    RSVD_FLAG_SHIFTED, RSVD_GAUSSIAN, RSVD_GSRFT, RSVD_MAX_L, RSVD_NATIVE, RSVD_SRFT, RsvdError, RsvdProblem,
)

PRECISIONS = {"native": RSVD_NATIVE, "bf16": RSVD_BF16, "bf16x3": RSVD_BF16X3}
SKETCHES = {"gaussian": RSVD_GAUSSIAN, "srft": RSVD_SRFT, "gsrft": RSVD_GSRFT}
_DTYPES = {torch.float32: RSVD_F32, torch.float64: RSVD_F64}


def problem(m, n, k, p, q=0, *, dtype=torch.float32, sketch="gaussian", prec="native", seed=0,
            stream_id=0, lda=None):
    """Build the C problem descriptor (a host struct)."""
    pr = RsvdProblem()
    pr.m, pr.n, pr.lda = int(m), int(n), int(lda if lda is not None else n)
    pr.k, pr.p, pr.q = int(k), int(p), int(q)
    pr.dtype = _DTYPES[dtype] if isinstance(dtype, torch.dtype) else int(dtype)
    pr.sketch = SKETCHES[sketch] if isinstance(sketch, str) else int(sketch)
    pr.prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    pr.seed, pr.stream_id = int(seed) & (2**64 - 1), int(stream_id) & (2**64 - 1)
    return pr


class Handle:
    """An rsvd_handle on one device (owns only the device status word)."""

    def __init__(self, device):
        self.lib = _lib.load()
        self.device = int(device)
        self.ptr = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self.lib.rsvd_create(ctypes.byref(self.ptr), self.device), "rsvd_create")

    def __del__(self):
        try:
            if self.ptr:
                self.lib.rsvd_destroy(self.ptr)
        except Exception:
            pass


_HANDLES = {}


def handle(device=None):
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    if idx not in _HANDLES:
        _HANDLES[idx] = Handle(idx)
    return _HANDLES[idx]


def validate(pr):
    return int(_lib.load().rsvd_validate(ctypes.byref(pr)))


def workspace_bytes(pr):
    return int(_lib.load().rsvd_workspace_bytes(ctypes.byref(pr)))


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_matrix(A, name="A"):
    if not A.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError(f"{name} must be a row-major 2-D tensor (unit column stride)")
    if A.dtype not in _DTYPES:
        raise ValueError(f"{name} must be float32 or float64")


def _elem_dtype(pr):
    return torch.float64 if pr.dtype == RSVD_F64 else torch.float32


class Workspace:
    """A caller-owned workspace buffer sized for a problem (torch allocation)."""

    def __init__(self, pr, device):
        nbytes = workspace_bytes(pr)
        if nbytes == 0:
            raise RsvdError(validate(pr) or _lib.RSVD_E_INVAL, "rsvd_workspace_bytes")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.nbytes = nbytes

    @property
    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr())


def _prob_for(A, k, p, q, sketch, prec, seed, stream_id):
    _check_matrix(A)
    m, n = A.shape
    return problem(m, n, k, p, q, dtype=A.dtype, sketch=sketch, prec=prec, seed=seed,
                   stream_id=stream_id, lda=A.stride(0))


def rsvd_range_finder(A, k, p, *, q=0, sketch="gaussian", prec="native", seed=0, stream_id=0,
                      Q=None, ws=None):
    pr = _prob_for(A, k, p, q, sketch, prec, seed, stream_id)
    l = k + p
    if Q is None:
        Q = torch.empty(A.shape[0], l, dtype=_elem_dtype(pr), device=A.device)
    ws = ws or Workspace(pr, A.device)
    h = handle(A.device)
    _lib.check(h.lib.rsvd_range_finder(h.ptr, ctypes.byref(pr), _ptr(A), _ptr(Q), ws.ptr, ws.nbytes,
                                       _stream(A.device)), "rsvd_range_finder")
    return Q


def rsvd_power_iter(A, Q, k, p, q, *, sketch="gaussian", prec="native", seed=0, stream_id=0, ws=None):
    pr = _prob_for(A, k, p, q, sketch, prec, seed, stream_id)
    ws = ws or Workspace(pr, A.device)
    h = handle(A.device)
    _lib.check(h.lib.rsvd_power_iter(h.ptr, ctypes.byref(pr), _ptr(A), _ptr(Q), ws.ptr, ws.nbytes,
                                     _stream(A.device)), "rsvd_power_iter")
    return Q


def rsvd_project(A, Q, k, p, *, q=0, sketch="gaussian", prec="native", seed=0, stream_id=0, Bt=None,
                 ws=None):
    pr = _prob_for(A, k, p, q, sketch, prec, seed, stream_id)
    if Bt is None:
        Bt = torch.empty(A.shape[1], k + p, dtype=Q.dtype, device=A.device)
    ws = ws or Workspace(pr, A.device)
    h = handle(A.device)
    _lib.check(h.lib.rsvd_project(h.ptr, ctypes.byref(pr), _ptr(A), _ptr(Q), _ptr(Bt), ws.ptr, ws.nbytes,
                                  _stream(A.device)), "rsvd_project")
    return Bt


def rsvd_svd(Bt, Q, m, n, k, p, *, q=0, dtype=torch.float32, sketch="gaussian", prec="native", seed=0,
             stream_id=0, U=None, S=None, V=None, ws=None):
    pr = problem(m, n, k, p, q, dtype=dtype, sketch=sketch, prec=prec, seed=seed, stream_id=stream_id)
    dev = Bt.device
    real = _elem_dtype(pr)
    if U is None:
        U = torch.empty(m, k, dtype=Q.dtype, device=dev)
    if S is None:
        S = torch.empty(k, dtype=real, device=dev)
    if V is None:
        V = torch.empty(n, k, dtype=Bt.dtype, device=dev)
    ws = ws or Workspace(pr, dev)
    h = handle(dev)
    _lib.check(h.lib.rsvd_svd(h.ptr, ctypes.byref(pr), _ptr(Bt), _ptr(Q), _ptr(U), _ptr(S), _ptr(V), ws.ptr,
                              ws.nbytes, _stream(dev)), "rsvd_svd")
    return U, S, V


def _herm(fn, A, Q, k, p, prec, U, Lam, ws):
    n = A.shape[0]
    if A.dim() != 2 or A.shape[1] != n:
        raise ValueError(f"{fn}: A must be square, got {tuple(A.shape)}")
    pr = problem(n, n, k, p, 0, dtype=A.dtype, prec=prec)
    dev = A.device
    if U is None:
        U = torch.empty(n, k, dtype=A.dtype, device=dev)
    if Lam is None:
        Lam = torch.empty(k, dtype=A.dtype, device=dev)
    ws = ws or Workspace(pr, dev)
    h = handle(dev)
    _lib.check(getattr(h.lib, fn)(h.ptr, ctypes.byref(pr), _ptr(A), _ptr(Q), _ptr(U), _ptr(Lam), ws.ptr,
                                  ws.nbytes, _stream(dev)), fn)
    return U, Lam


def rsvd_eigh(A, Q, k, *, prec="native", U=None, Lam=None, ws=None):
    """Algorithm 5.3 for symmetric A (n x n) and a basis Q (n x l, l = Q.shape[1] >= k): the k
    eigenpairs of largest |lambda| of Q^T A Q, lifted by Q.  Returns (U (n x k), Lam (k,))."""
    return _herm("rsvd_eigh", A, Q, k, Q.shape[1] - k, prec, U, Lam, ws)


def rsvd_nystrom(A, Q, k, *, prec="native", U=None, Lam=None, ws=None):
    """Algorithm 5.5 (Nystrom) for positive semidefinite A (n x n) and a basis Q (n x l):
    returns (U (n x k), Lam (k,)) with U Lam U^T the rank-k part of (AQ)(Q^T A Q)^-1 (AQ)^T."""
    return _herm("rsvd_nystrom", A, Q, k, Q.shape[1] - k, prec, U, Lam, ws)


def rsvd_eigh_onepass(A, k, p=10, *, prec="native", seed=0, stream_id=0, U=None, Lam=None, ws=None):
    """Algorithm 5.6 for symmetric A (n x n): one pass over A (Y = A Omega, Omega n x (k + p) from
    (seed, stream_id)), B from the least-squares system B (Q^T Omega) = Q^T Y, its eigenpairs lifted by
    Q.  Returns (U (n x k), Lam (k,)) in decreasing |lambda|."""
    n = A.shape[0]
    if A.dim() != 2 or A.shape[1] != n:
        raise ValueError(f"rsvd_eigh_onepass: A must be square, got {tuple(A.shape)}")
    pr = problem(n, n, k, p, 0, dtype=A.dtype, prec=prec, seed=seed, stream_id=stream_id)
    dev = A.device
    if U is None:
        U = torch.empty(n, k, dtype=A.dtype, device=dev)
    if Lam is None:
        Lam = torch.empty(k, dtype=A.dtype, device=dev)
    ws = ws or Workspace(pr, dev)
    h = handle(dev)
    _lib.check(h.lib.rsvd_eigh_onepass(h.ptr, ctypes.byref(pr), _ptr(A), _ptr(U), _ptr(Lam), ws.ptr, ws.nbytes,
                                       _stream(dev)), "rsvd_eigh_onepass")
    return U, Lam


def rsvd_svd_onepass(A, k, p=10, *, prec="native", seed=0, stream_id=0, U=None, S=None, V=None, ws=None):
    """The single-pass factorization of a general A (Section 5.5): Y = A Omega and Yt = A^T Omegat,
    bases Q and Qt, B from its two least-squares relations, B = Ub S Vb^T.  Returns (U (m x k), S (k,),
    V (n x k))."""
    m, n = A.shape
    pr = problem(m, n, k, p, 0, dtype=A.dtype, prec=prec, seed=seed, stream_id=stream_id)
    dev = A.device
    U = torch.empty(m, k, dtype=A.dtype, device=dev) if U is None else U
    S = torch.empty(k, dtype=A.dtype, device=dev) if S is None else S
    V = torch.empty(n, k, dtype=A.dtype, device=dev) if V is None else V
    ws = ws or Workspace(pr, dev)
    h = handle(dev)
    _lib.check(h.lib.rsvd_svd_onepass(h.ptr, ctypes.byref(pr), _ptr(A), _ptr(U), _ptr(S), _ptr(V), ws.ptr,
                                      ws.nbytes, _stream(dev)), "rsvd_svd_onepass")
    return U, S, V


def _check_differentiable(sketch):
    """The adjoint holds the test matrix fixed as an explicit Omega: only the Gaussian sketch
    has one (the SRFT's Omega is applied implicitly by FFTs).  Refused like the C ABI's
    rsvd_backward_workspace_bytes refuses it, rather than silently switching sketches."""
    name = sketch if isinstance(sketch, str) else {v: k for k, v in SKETCHES.items()}.get(int(sketch), sketch)
    if name != "gaussian":
        raise RsvdError(_lib.RSVD_E_UNSUPPORTED,
                        f"rsvd under autograd: the adjoint supports the Gaussian sketch only (got {name!r})")


def rsvd(A, k, p=10, q=0, *, sketch="gaussian", prec="native", seed=0, stream_id=0, ws=None,
         return_q=False, keep_state=False):
    """Randomized SVD of A: the four entry points in sequence.  Returns (U, S, V).

    When A requires grad (and grad mode is on) the result is differentiable
    through RSVDFunction.  By default its backward is rsvd_backward, which
    recomputes the forward (nothing but A is held between the two passes);
    keep_state=True instead runs rsvd_forward_kept / rsvd_backward_kept, which
    hold every basis of the power scheme, (q + 1) m l + q n l elements plus the
    l x l factors, from the forward to the backward to skip the recomputation.
    Only the Gaussian sketch is differentiable (RsvdError otherwise).
    """
    if A.requires_grad and torch.is_grad_enabled() and not return_q:
        _check_differentiable(sketch)
        return RSVDFunction.apply(A, k, p, q, seed, stream_id, prec, bool(keep_state))
    pr = _prob_for(A, k, p, q, sketch, prec, seed, stream_id)
    ws = ws or Workspace(pr, A.device)
    kw = dict(sketch=sketch, prec=prec, seed=seed, stream_id=stream_id, ws=ws)
    Q = rsvd_range_finder(A, k, p, q=q, **kw)
    rsvd_power_iter(A, Q, k, p, q, **kw)
    Bt = rsvd_project(A, Q, k, p, q=q, **kw)
    m, n = A.shape
    U, S, V = rsvd_svd(Bt, Q, m, n, k, p, q=q, dtype=A.dtype, **kw)
    if return_q:
        return U, S, V, Q, Bt
    return U, S, V


def full_workspace(pr, device):
    """A workspace for rsvd_full (torch allocation): Q, Bt and the hot-path workspace."""
    nbytes = handle(device).lib.rsvd_full_workspace_bytes(ctypes.byref(pr))
    if nbytes == 0:
        raise RsvdError(validate(pr) or _lib.RSVD_E_INVAL, "rsvd_full_workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def rsvd_full(A, k, p=10, q=0, *, sketch="gaussian", prec="native", seed=0, stream_id=0, outs=None, ws=None):
    """(U, S, V): the four hot-path calls as one, replayed from a HIP graph when `outs` (a previous
    return value) and `ws` (from full_workspace) are passed back with the same A."""
    pr = _prob_for(A, k, p, q, sketch, prec, seed, stream_id)
    dev = A.device
    ws = full_workspace(pr, dev) if ws is None else ws
    if outs is None:
        m, n = A.shape
        outs = (torch.empty(m, k, dtype=A.dtype, device=dev), torch.empty(k, dtype=A.dtype, device=dev),
                torch.empty(n, k, dtype=A.dtype, device=dev))
    U, S, V = outs
    h = handle(dev)
    _lib.check(h.lib.rsvd_full(h.ptr, ctypes.byref(pr), _ptr(A), _ptr(U), _ptr(S), _ptr(V),
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev)), "rsvd_full")
    return U, S, V


def rsvd_full_static(A, k, p=10, q=0, *, sketch="gaussian", prec="native", seed=0, stream_id=0, outs=None):
    """(U, S, V) = rsvd_full with the library's static device workspace: no workspace argument
    and no allocation inside the call (the outputs are allocated here unless `outs` is given).
    Problems whose rsvd_full workspace exceeds RSVD_STATIC_SCRATCH_BYTES raise RsvdError."""
    pr = _prob_for(A, k, p, q, sketch, prec, seed, stream_id)
    dev = A.device
    if outs is None:
        m, n = A.shape
        outs = (torch.empty(m, k, dtype=A.dtype, device=dev), torch.empty(k, dtype=A.dtype, device=dev),
                torch.empty(n, k, dtype=A.dtype, device=dev))
    U, S, V = outs
    h = handle(dev)
    _lib.check(h.lib.rsvd_full_static(h.ptr, ctypes.byref(pr), _ptr(A), _ptr(U), _ptr(S), _ptr(V), _stream(dev)),
               "rsvd_full_static")
    return U, S, V


def rsvd_range_finder_tol(A, eps, b0=16, lmax=128, r=10, *, prec="native", seed=0, stream_id=0, Q=None):
    """Fixed-precision range finder (Algorithm 4.2 in blocks b0, b0, 2 b0, ... up to lmax): returns
    (Q[:, :l], l, est) with est the a posteriori estimate of ||(I - Q Q*) A|| of eq. (4.3); est <= eps
    unless the capacity lmax was reached first.  Synchronizes the current stream."""
    pr = _prob_for(A, b0, lmax - b0, 0, "gaussian", prec, seed, stream_id)
    lib = _lib.load()
    nbytes = int(lib.rsvd_range_finder_tol_workspace_bytes(ctypes.byref(pr), int(r)))
    if nbytes == 0:
        raise RsvdError(validate(pr) or _lib.RSVD_E_INVAL, "rsvd_range_finder_tol_workspace_bytes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    if Q is None:
        Q = torch.zeros(A.shape[0], lmax, dtype=_elem_dtype(pr), device=A.device)
    l_out = ctypes.c_int32(0)
    est = ctypes.c_double(0.0)
    h = handle(A.device)
    _lib.check(h.lib.rsvd_range_finder_tol(h.ptr, ctypes.byref(pr), float(eps), int(r), _ptr(A), _ptr(Q),
                                           ctypes.byref(l_out), ctypes.byref(est), ctypes.c_void_p(ws.data_ptr()),
                                           nbytes, _stream(A.device)), "rsvd_range_finder_tol")
    return Q[:, :l_out.value], int(l_out.value), float(est.value)


def rsvd_sketch(A, k, p, *, sketch="gaussian", prec="native", seed=0, stream_id=0, Y=None, ws=None):
    """Y = A Omega (m x (k+p)) with the test matrix the range finder draws, not orthonormalized."""
    pr = _prob_for(A, k, p, 0, sketch, prec, seed, stream_id)
    if Y is None:
        Y = torch.empty(A.shape[0], k + p, dtype=_elem_dtype(pr), device=A.device)
    ws = ws or Workspace(pr, A.device)
    h = handle(A.device)
    _lib.check(h.lib.rsvd_sketch(h.ptr, ctypes.byref(pr), _ptr(A), _ptr(Y), ws.ptr, ws.nbytes, _stream(A.device)),
               "rsvd_sketch")
    return Y


def backward_workspace(pr, device):
    """A workspace for the adjoint calls of one problem (torch allocation)."""
    nbytes = handle(device).lib.rsvd_backward_workspace_bytes(ctypes.byref(pr))
    if nbytes == 0:
        raise RsvdError(validate(pr) or _lib.RSVD_E_UNSUPPORTED, "rsvd_backward_workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _adjoint_call(fn, A, gU, gS, gV, pr, ws, gA):
    dev = A.device
    h = handle(dev)
    gU, gS, gV = (t.detach().to(A.dtype).contiguous() for t in (gU, gS, gV))
    if gA is None:
        gA = torch.empty(A.shape, dtype=A.dtype, device=dev)
    _lib.check(getattr(h.lib, fn)(h.ptr, ctypes.byref(pr), _ptr(A), _ptr(gU), _ptr(gS), _ptr(gV), _ptr(gA),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev)), fn)
    return gA


def rsvd_backward(A, gU, gS, gV, k, p, q, *, prec="native", seed=0, stream_id=0, gA=None, ws=None):
    """gA = the adjoint of A -> (U, S, V) applied to (gU, gS, gV) (fixed test matrix); the
    forward is recomputed inside."""
    pr = _prob_for(A, k, p, q, "gaussian", prec, seed, stream_id)
    ws = backward_workspace(pr, A.device) if ws is None else ws
    return _adjoint_call("rsvd_backward", A, gU, gS, gV, pr, ws, gA)


def rsvd_forward_kept(A, k, p, q, *, prec="native", seed=0, stream_id=0, ws=None):
    """(U, S, V, ws): the randomized SVD computed in an adjoint workspace that keeps the
    forward state for rsvd_backward_kept."""
    pr = _prob_for(A, k, p, q, "gaussian", prec, seed, stream_id)
    dev = A.device
    ws = backward_workspace(pr, dev) if ws is None else ws
    m, n = A.shape
    U = torch.empty(m, k, dtype=A.dtype, device=dev)
    S = torch.empty(k, dtype=A.dtype, device=dev)
    V = torch.empty(n, k, dtype=A.dtype, device=dev)
    h = handle(dev)
    _lib.check(h.lib.rsvd_forward_kept(h.ptr, ctypes.byref(pr), _ptr(A), _ptr(U), _ptr(S), _ptr(V),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev)), "rsvd_forward_kept")
    return U, S, V, ws


def rsvd_backward_kept(A, gU, gS, gV, k, p, q, ws, *, prec="native", seed=0, stream_id=0, gA=None):
    """rsvd_backward from the state rsvd_forward_kept left in `ws` (same problem, same A)."""
    pr = _prob_for(A, k, p, q, "gaussian", prec, seed, stream_id)
    return _adjoint_call("rsvd_backward_kept", A, gU, gS, gV, pr, ws, gA)


class RSVDFunction(torch.autograd.Function):
    """(U, S, V) = rsvd(A) with the library's hand-written adjoint as backward.

    keep_state False (the default): the forward is the four hot-path calls and the backward
    is rsvd_backward, which recomputes the forward's bases from A and the fixed test matrix.
    keep_state True: the forward keeps its state (rsvd_forward_kept) and the backward is
    rsvd_backward_kept; gA is the same either way."""

    @staticmethod
    def forward(ctx, A, k, p, q, seed, stream_id, prec, keep_state=False):
        Ad = A.detach()
        if keep_state:
            U, S, V, ws = rsvd_forward_kept(Ad, k, p, q, prec=prec, seed=seed, stream_id=stream_id)
            ctx.save_for_backward(Ad, ws)
        else:
            U, S, V = rsvd(Ad, k, p, q, prec=prec, seed=seed, stream_id=stream_id)
            ctx.save_for_backward(Ad)
        ctx.cfg = (k, p, q, seed, stream_id, prec, keep_state)
        return U, S, V

    @staticmethod
    def backward(ctx, gU, gS, gV):
        k, p, q, seed, stream_id, prec, keep_state = ctx.cfg
        A = ctx.saved_tensors[0]
        m, n = A.shape
        z = lambda shape: torch.zeros(shape, dtype=A.dtype, device=A.device)
        gU = z((m, k)) if gU is None else gU
        gS = z((k,)) if gS is None else gS
        gV = z((n, k)) if gV is None else gV
        if keep_state:
            gA = rsvd_backward_kept(A, gU, gS, gV, k, p, q, ctx.saved_tensors[1], prec=prec, seed=seed,
                                    stream_id=stream_id)
        else:
            gA = rsvd_backward(A, gU, gS, gV, k, p, q, prec=prec, seed=seed, stream_id=stream_id)
        return gA, None, None, None, None, None, None, None


class BatchWorkspace:
    """A caller-owned workspace for rsvd_batched (torch allocation)."""

    def __init__(self, probs, device):
        arr = (RsvdProblem * len(probs))(*probs)
        h = handle(device)
        nbytes = h.lib.rsvd_batched_workspace_bytes(len(probs), arr)
        if nbytes == 0:
            raise RsvdError(_lib.RSVD_E_INVAL, "rsvd_batched_workspace_bytes")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.nbytes = nbytes

    @property
    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr())


def _batch_problems(As, ks, p, q, prec, seed, stream_id):
    count = len(As)
    ks = [int(ks)] * count if isinstance(ks, int) else [int(k) for k in ks]
    if len(ks) != count:
        raise ValueError("one rank per matrix")
    dev = As[0].device
    probs = []
    for i, (A, k) in enumerate(zip(As, ks)):
        _check_matrix(A)
        if A.dtype != As[0].dtype or A.device != dev:
            raise ValueError("all matrices must share dtype and device")
        m, n = A.shape
        probs.append(problem(m, n, k, p, q, dtype=A.dtype, prec=prec, seed=seed, stream_id=stream_id + i,
                             lda=A.stride(0)))
    return ks, probs


def _ptrs(ts):
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


def rsvd_batched(As, ks, p=8, q=1, *, prec="native", seed=0, stream_id=0, outs=None, ws=None,
                 keep_state=False):
    """Randomized SVDs of many independent matrices in one batched call.

    As: list of 2-D CUDA tensors (same dtype), ks: target ranks (int or list).
    Matrix i draws its test matrix from (seed, stream_id + i).  Returns a list
    of (U, S, V).  `outs` (a previous return value) and `ws` (a BatchWorkspace)
    may be passed back to reuse buffers, which lets the library replay its
    recorded graph without re-pointing it.  When any matrix requires grad (and
    grad mode is on) the result is differentiable through
    RSVDBatchedFunction, whose backward is rsvd_backward_batched (the forward
    recomputed); keep_state=True holds every problem's forward state instead
    (rsvd_batched_kept / rsvd_backward_batched_kept).
    """
    count = len(As)
    if count == 0:
        return []
    if torch.is_grad_enabled() and any(A.requires_grad for A in As):
        flat = RSVDBatchedFunction.apply((ks, p, q, prec, seed, stream_id, bool(keep_state)), *As)
        return [tuple(flat[3 * i:3 * i + 3]) for i in range(count)]
    ks, probs = _batch_problems(As, ks, p, q, prec, seed, stream_id)
    dev = As[0].device
    if outs is None:
        outs = [(torch.empty(A.shape[0], k, dtype=A.dtype, device=dev), torch.empty(k, dtype=A.dtype, device=dev),
                 torch.empty(A.shape[1], k, dtype=A.dtype, device=dev)) for A, k in zip(As, ks)]
    ws = ws or BatchWorkspace(probs, dev)
    arr = (RsvdProblem * count)(*probs)
    h = handle(dev)
    _lib.check(h.lib.rsvd_batched(h.ptr, count, arr, _ptrs(As), _ptrs([o[0] for o in outs]),
                                  _ptrs([o[1] for o in outs]), _ptrs([o[2] for o in outs]), ws.ptr, ws.nbytes,
                                  _stream(dev)), "rsvd_batched")
    return outs


def backward_batched_workspace(probs, device):
    """A workspace for the batched adjoint calls (torch allocation)."""
    arr = (RsvdProblem * len(probs))(*probs)
    nbytes = handle(device).lib.rsvd_backward_batched_workspace_bytes(len(probs), arr)
    if nbytes == 0:
        raise RsvdError(_lib.RSVD_E_INVAL, "rsvd_backward_batched_workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _batched_adjoint_call(fn, As, gUs, gSs, gVs, probs, ws, gAs):
    dev = As[0].device
    h = handle(dev)
    gUs, gSs, gVs = ([t.detach().to(As[0].dtype).contiguous() for t in ts] for ts in (gUs, gSs, gVs))
    if gAs is None:
        gAs = [torch.empty(A.shape, dtype=A.dtype, device=dev) for A in As]
    arr = (RsvdProblem * len(As))(*probs)
    _lib.check(getattr(h.lib, fn)(h.ptr, len(As), arr, _ptrs(As), _ptrs(gUs), _ptrs(gSs), _ptrs(gVs), _ptrs(gAs),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev)), fn)
    return gAs


def rsvd_backward_batched(As, gUs, gSs, gVs, ks, p, q, *, prec="native", seed=0, stream_id=0, gAs=None, ws=None):
    """gA_i = the adjoint of A_i -> (U_i, S_i, V_i) applied to (gU_i, gS_i, gV_i) for every
    matrix of a batch (fixed test matrices, matrix i drawing from (seed, stream_id + i)); the
    forward is recomputed inside."""
    if len(As) == 0:
        return []
    ks, probs = _batch_problems(As, ks, p, q, prec, seed, stream_id)
    ws = backward_batched_workspace(probs, As[0].device) if ws is None else ws
    return _batched_adjoint_call("rsvd_backward_batched", As, gUs, gSs, gVs, probs, ws, gAs)


def rsvd_batched_kept(As, ks, p=8, q=1, *, prec="native", seed=0, stream_id=0, ws=None):
    """(outs, ws): rsvd_batched computed in a batched adjoint workspace that keeps every
    problem's forward state for rsvd_backward_batched_kept."""
    ks, probs = _batch_problems(As, ks, p, q, prec, seed, stream_id)
    dev = As[0].device
    ws = backward_batched_workspace(probs, dev) if ws is None else ws
    outs = [(torch.empty(A.shape[0], k, dtype=A.dtype, device=dev), torch.empty(k, dtype=A.dtype, device=dev),
             torch.empty(A.shape[1], k, dtype=A.dtype, device=dev)) for A, k in zip(As, ks)]
    arr = (RsvdProblem * len(As))(*probs)
    h = handle(dev)
    _lib.check(h.lib.rsvd_batched_kept(h.ptr, len(As), arr, _ptrs(As), _ptrs([o[0] for o in outs]),
                                       _ptrs([o[1] for o in outs]), _ptrs([o[2] for o in outs]),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev)), "rsvd_batched_kept")
    return outs, ws


def rsvd_backward_batched_kept(As, gUs, gSs, gVs, ks, p, q, ws, *, prec="native", seed=0, stream_id=0, gAs=None):
    """rsvd_backward_batched from the state rsvd_batched_kept left in `ws`."""
    ks, probs = _batch_problems(As, ks, p, q, prec, seed, stream_id)
    return _batched_adjoint_call("rsvd_backward_batched_kept", As, gUs, gSs, gVs, probs, ws, gAs)


class RSVDBatchedFunction(torch.autograd.Function):
    """Flat (U_0, S_0, V_0, U_1, ...) = rsvd_batched(As).  By default the forward is
    rsvd_batched and the backward rsvd_backward_batched (the forward recomputed); with
    keep_state the forward keeps its state (rsvd_batched_kept) and the backward is
    rsvd_backward_batched_kept."""

    @staticmethod
    def forward(ctx, cfg, *As):
        ks, p, q, prec, seed, stream_id, keep_state = cfg
        Ad = [A.detach() for A in As]
        if keep_state:
            outs, ws = rsvd_batched_kept(Ad, ks, p, q, prec=prec, seed=seed, stream_id=stream_id)
            ctx.save_for_backward(ws, *Ad)
        else:
            outs = rsvd_batched(Ad, ks, p, q, prec=prec, seed=seed, stream_id=stream_id)
            ctx.save_for_backward(*Ad)
        ctx.cfg = ([o[1].shape[0] for o in outs], p, q, prec, seed, stream_id, keep_state)
        return tuple(t for o in outs for t in o)

    @staticmethod
    def backward(ctx, *grads):
        ks, p, q, prec, seed, stream_id, keep_state = ctx.cfg
        if keep_state:
            ws, *As = ctx.saved_tensors
        else:
            ws, As = None, list(ctx.saved_tensors)
        gUs, gSs, gVs = [], [], []
        for i, (A, k) in enumerate(zip(As, ks)):
            m, n = A.shape
            gU, gS, gV = grads[3 * i:3 * i + 3]
            z = lambda shape: torch.zeros(shape, dtype=A.dtype, device=A.device)
            gUs.append(z((m, k)) if gU is None else gU)
            gSs.append(z((k,)) if gS is None else gS)
            gVs.append(z((n, k)) if gV is None else gV)
        if keep_state:
            gAs = rsvd_backward_batched_kept(As, gUs, gSs, gVs, ks, p, q, ws, prec=prec, seed=seed,
                                             stream_id=stream_id)
        else:
            gAs = rsvd_backward_batched(As, gUs, gSs, gVs, ks, p, q, prec=prec, seed=seed, stream_id=stream_id)
        return (None, *gAs)


def rsvd_draw_omega(n, k, p, *, dtype=torch.float32, seed=0, stream_id=0, device="cuda"):
    """The Gaussian test matrix the range finder draws (n x (k+p))."""
    pr = problem(max(n, k + p), n, k, p, 0, dtype=dtype, seed=seed, stream_id=stream_id)
    Om = torch.empty(n, k + p, dtype=dtype, device=device)
    h = handle(Om.device)
    _lib.check(h.lib.rsvd_draw_omega(h.ptr, ctypes.byref(pr), _ptr(Om), _stream(Om.device)), "rsvd_draw_omega")
    return Om


def rsvd_draw_srft(n, k, p, *, dtype=torch.float32, seed=0, stream_id=0, device="cuda"):
    """The SRFT ingredients the range finder draws: signs d (n, float64) and frequencies R (k+p, int32)."""
    pr = problem(max(n, k + p), n, k, p, 0, dtype=dtype, sketch="srft", seed=seed, stream_id=stream_id)
    d = torch.empty(n, dtype=torch.float64, device=device)
    R = torch.empty(k + p, dtype=torch.int32, device=device)
    h = handle(d.device)
    _lib.check(h.lib.rsvd_draw_srft(h.ptr, ctypes.byref(pr), _ptr(d), _ptr(R), _stream(d.device)),
               "rsvd_draw_srft")
    return d, R


def rsvd_orth(Y, want_r=True, ws=None):
    """CholeskyQR2 of a tall Y (in place): returns (Q, R)."""
    _check_matrix(Y, "Y")
    rows, l = Y.shape
    if Y.stride(0) != l:
        raise ValueError("Y must be contiguous")
    pr = problem(rows, l, l, 0, 0, dtype=Y.dtype)
    ws = ws or Workspace(pr, Y.device)
    R = torch.empty(l, l, dtype=torch.float64, device=Y.device) if want_r else None
    h = handle(Y.device)
    _lib.check(h.lib.rsvd_orth(h.ptr, ctypes.byref(pr), rows, _ptr(Y), _ptr(R), ws.ptr, ws.nbytes,
                               _stream(Y.device)), "rsvd_orth")
    return Y, R


def device_status(device=None):
    """Synchronize and return (and clear) the handle's RSVD_FLAG_* bits."""
    h = handle(device)
    flags = ctypes.c_int32(0)
    dev = torch.device("cuda", h.device)
    _lib.check(h.lib.rsvd_device_status(h.ptr, _stream(dev), ctypes.byref(flags)), "rsvd_device_status")
    return int(flags.value)


def profile_enable(capacity, device=None):
    """Time every launch of the library's kernel families with HIP events (capacity launches)."""
    h = handle(device)
    _lib.check(h.lib.rsvd_profile_enable(h.ptr, int(capacity)), "rsvd_profile_enable")


def profile_select(families, device=None):
    """Time only the named kernel families (see _lib.KERNEL_KINDS) until the next profile_enable."""
    h = handle(device)
    mask = 0
    for f in families:
        mask |= 1 << _lib.KERNEL_KINDS.index(f)
    _lib.check(h.lib.rsvd_profile_select(h.ptr, mask), "rsvd_profile_select")


def profile_read(device=None):
    """{family: (launches, total_ms)} since the last read; waits for the events."""
    h = handle(device)
    n = len(_lib.KERNEL_KINDS)
    launches = (ctypes.c_int32 * n)()
    ms = (ctypes.c_double * n)()
    _lib.check(h.lib.rsvd_profile_read(h.ptr, launches, ms), "rsvd_profile_read")
    return {name: (int(launches[i]), float(ms[i])) for i, name in enumerate(_lib.KERNEL_KINDS)}


MFMA_PROBE_FLOPS = {"bf16": 32768, "fp32": 4096, "fp64": 2048}


def probe_hbm_read(buf):
    """Enqueue the library's streaming-read probe over the device tensor `buf` (a measurement aid:
    the caller times it on the current stream).  Returns the sink tensor."""
    nbytes = buf.numel() * buf.element_size() // 16 * 16
    sink = torch.empty(2048, dtype=torch.float32, device=buf.device)
    _lib.check(_lib.load().rsvd_probe_hbm_read(_ptr(buf), nbytes, _ptr(sink), _stream(buf.device)),
               "rsvd_probe_hbm_read")
    return sink, nbytes


def probe_mfma(kind, iters, blocks, device=None):
    """Enqueue the library's MFMA-loop probe (kind "bf16", "fp32" or "fp64"); returns (sink, flops)."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    k = {"bf16": 0, "fp32": 1, "fp64": 2}[kind]
    sink = torch.empty(int(blocks) * 256, dtype=torch.float32, device=dev)
    _lib.check(_lib.load().rsvd_probe_mfma(k, int(iters), int(blocks), _ptr(sink), _stream(dev)), "rsvd_probe_mfma")
    return sink, float(blocks) * 4 * 4 * float(iters) * MFMA_PROBE_FLOPS[kind]
