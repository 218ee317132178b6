"""Reference gradient of the fixed-Omega randomized SVD, in FP64 on the CPU.

TEST INFRASTRUCTURE (see the package docstring): only tests and the smoke
check use this module.

The paper defines the forward map (Algorithm 4.4 for Stage A, Algorithm 5.1
and the truncation remark of Section 5.1 for Stage B) and no derivative.  The
reference derivative here is that forward map written once more with plain
PyTorch CPU operations in FP64 -- the QR (Householder, then the column signs
that make diag(R) positive) and the SVD of the small matrix from
torch.linalg -- differentiated by torch.autograd.  The test matrix Omega is
an input (drawn by oracle.philox), held fixed.

A loss that depends on the factors only through U_k diag(S_k) V_k^T and S_k
does not depend on the sign (phase) choices of the singular vectors or of
the basis Q, so its gradient with respect to A is well defined and can be
compared between implementations that choose signs differently.
"""

import numpy as np
import torch


def qr_pos(Y):
    """Thin QR with diag(R) > 0 (Householder through torch.linalg.qr, then sign flips)."""
    Q, R = torch.linalg.qr(Y, mode="reduced")
    d = torch.sign(torch.diagonal(R))
    d = torch.where(d == 0, torch.ones_like(d), d)
    return Q * d[None, :]


def rsvd_torch(A, k, p, q, Omega):
    """(U_k, S_k, V_k) of Algorithm 4.4 + Algorithm 5.1 with the given Omega, differentiable in A."""
    Q = qr_pos(A @ Omega)
    for _ in range(q):
        Qt = qr_pos(A.T @ Q)
        Q = qr_pos(A @ Qt)
    B = Q.T @ A
    Ut, S, Vh = torch.linalg.svd(B, full_matrices=False)
    U = Q @ Ut
    return U[:, :k], S[:k], Vh.T[:, :k]


def reconstruction_loss(U, S, V, T, w):
    """||U diag(S) V^T - T||_F^2 + sum_i w_i S_i (invariant to sign choices)."""
    return ((U * S[None, :]) @ V.T - T).square().sum() + (w * S).sum()


def loss_and_grad(A, k, p, q, Omega, T, w):
    """The loss above and its gradient with respect to A, in FP64 (numpy in, numpy out)."""
    At = torch.tensor(np.asarray(A, dtype=np.float64), requires_grad=True)
    Om = torch.tensor(np.asarray(Omega, dtype=np.float64))
    Tt = torch.tensor(np.asarray(T, dtype=np.float64))
    wt = torch.tensor(np.asarray(w, dtype=np.float64))
    U, S, V = rsvd_torch(At, k, p, q, Om)
    L = reconstruction_loss(U, S, V, Tt, wt)
    L.backward()
    return float(L.detach()), At.grad.numpy()


def loss_value(A, k, p, q, Omega, T, w):
    with torch.no_grad():
        At = torch.tensor(np.asarray(A, dtype=np.float64))
        U, S, V = rsvd_torch(At, k, p, q, torch.tensor(np.asarray(Omega, dtype=np.float64)))
        return float(reconstruction_loss(U, S, V, torch.tensor(np.asarray(T, dtype=np.float64)),
                                         torch.tensor(np.asarray(w, dtype=np.float64))))
