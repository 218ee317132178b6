"""Residual norms and the paper's error bounds, in FP64.

TEST INFRASTRUCTURE (see the package docstring): only tests, the smoke check
and the benchmark's CPU-baseline leg use this module.

The approximation error of a basis Q is ||(I - QQ*) A|| (Section 1.3, the
fixed-rank problem); the error of a factorization is ||A - U S V*||.  Both are
spectral norms.  Small problems take them from a dense SVD of the residual;
larger ones from ARPACK's largest singular value of the residual applied as an
operator, never formed.
"""

import numpy as np

DENSE_LIMIT = 4_000_000  # entries; below this the residual is formed and SVD'd


def _spectral_norm_operator(matvec, rmatvec, shape, dtype):
    from scipy.sparse.linalg import LinearOperator, svds

    op = LinearOperator(shape, matvec=matvec, rmatvec=rmatvec, dtype=dtype)
    rng = np.random.default_rng(12345)
    v0 = rng.standard_normal(min(shape))
    s = svds(op, k=1, which="LM", return_singular_vectors=False, tol=1e-12,
             v0=v0, maxiter=10_000)
    return float(s[0])


def spectral_norm(M):
    """||M||_2 of a dense matrix by its largest singular value (LAPACK)."""
    return float(np.linalg.svd(np.asarray(M), compute_uv=False)[0])


def residual_q(A, Q):
    """||A - Q (Q* A)||_2: the quantity the range finder controls (eq. for the fixed-rank problem)."""
    A = np.asarray(A)
    Q = np.asarray(Q)
    B = np.conj(Q).T @ A
    if A.size <= DENSE_LIMIT:
        return spectral_norm(A - Q @ B)
    dt = np.result_type(A, Q)
    Bh = np.conj(B).T
    Qh = np.conj(Q).T
    return _spectral_norm_operator(
        lambda x: A @ x - Q @ (B @ x),
        lambda y: np.conj(A).T @ y - Bh @ (Qh @ y),
        A.shape, dt)


def residual_usv(A, U, S, V):
    """||A - U diag(S) V*||_2: the error of a (truncated) factorization."""
    A = np.asarray(A)
    U = np.asarray(U)
    V = np.asarray(V)
    S = np.asarray(S)
    if A.size <= DENSE_LIMIT:
        return spectral_norm(A - (U * S[None, :]) @ np.conj(V).T)
    dt = np.result_type(A, U, V)
    Vh = np.conj(V).T
    Uh = np.conj(U).T
    Sc = S.reshape(-1, 1)

    def mv(x):
        x2 = x.reshape(A.shape[1], -1)
        return (A @ x2 - U @ (Sc * (Vh @ x2))).reshape(x.shape[:-1] + (A.shape[0],) if x.ndim == 1 else (A.shape[0], -1))

    def rmv(y):
        y2 = y.reshape(A.shape[0], -1)
        return (np.conj(A).T @ y2 - V @ (Sc * (Uh @ y2))).reshape((A.shape[1],) if y.ndim == 1 else (A.shape[1], -1))

    return _spectral_norm_operator(mv, rmv, A.shape, dt)


def orthonormality_error(Q):
    """max |Q*Q - I|, entrywise."""
    Q = np.asarray(Q)
    G = np.conj(Q).T @ Q
    return float(np.max(np.abs(G - np.eye(G.shape[0]))))


# ---------------------------------------------------------------------------
# Error bounds (Part III).  sigma is the full singular spectrum, descending,
# sigma[0] = sigma_1.
# ---------------------------------------------------------------------------

def _tail(sigma, k, power=1.0):
    s = np.asarray(sigma, dtype=np.float64)
    return float(np.sqrt(np.sum(s[k:] ** (2 * power))))


def thm9_1_bound(sigma, V, Omega, k):
    """Theorem 9.1 (deterministic error bound), spectral form, for one Omega.

    With A = U Sigma V* partitioned after k singular values, Omega1 = V1* Omega
    and Omega2 = V2* Omega:
        ||(I - P_Y) A||^2 <= ||Sigma2||^2 + ||Sigma2 Omega2 Omega1^+||^2,
    valid when Omega1 has full row rank.  V is the full n x n right factor.
    Returns the square root of the right-hand side.
    """
    sigma = np.asarray(sigma, dtype=np.float64)
    V = np.asarray(V)
    O1 = np.conj(V[:, :k]).T @ Omega
    O2 = np.conj(V[:, k:]).T @ Omega
    S2 = sigma[k:V.shape[1]]
    term = (S2[:, None] * O2) @ np.linalg.pinv(O1)
    s2 = S2[0] if S2.size else 0.0
    return float(np.sqrt(s2 ** 2 + spectral_norm(term) ** 2)) if term.size else float(s2)


def thm9_3_bound(sigma, k, res_q):
    """Theorem 9.3 (truncated SVD): ||A - A_hat_(k)|| <= sigma_{k+1} + ||(I - P_Z) A||."""
    return float(np.asarray(sigma)[k] + res_q)


def thm10_5_bound(sigma, k, p):
    """Theorem 10.5: E||(I - P_Y)A||_F <= (1 + k/(p-1))^{1/2} (sum_{j>k} sigma_j^2)^{1/2}."""
    return float(np.sqrt(1.0 + k / (p - 1.0)) * _tail(sigma, k))


def thm10_6_bound(sigma, k, p):
    """Theorem 10.6: E||(I - P_Y)A|| <= (1 + sqrt(k/(p-1))) sigma_{k+1} + e sqrt(k+p)/p * tail_F."""
    s = np.asarray(sigma, dtype=np.float64)
    return float((1.0 + np.sqrt(k / (p - 1.0))) * s[k]
                 + np.e * np.sqrt(k + p) / p * _tail(s, k))


def cor10_9_bound(sigma, k, p, form=1):
    """Corollary 10.9, simplified deviation bounds (p >= 4).

    form 1: (1 + 17 sqrt(1 + k/p)) sigma_{k+1} + 8 sqrt(k+p)/(p+1) tail_F,
            failure probability at most 6 e^{-p};
    form 2: (1 + 8 sqrt((k+p) p log p)) sigma_{k+1} + 3 sqrt(k+p) tail_F,
            failure probability at most 6 p^{-p}.
    """
    s = np.asarray(sigma, dtype=np.float64)
    if form == 1:
        return float((1.0 + 17.0 * np.sqrt(1.0 + k / p)) * s[k]
                     + 8.0 * np.sqrt(k + p) / (p + 1.0) * _tail(s, k))
    return float((1.0 + 8.0 * np.sqrt((k + p) * p * np.log(p))) * s[k]
                 + 3.0 * np.sqrt(k + p) * _tail(s, k))


def cor10_10_bound(sigma, k, p, q):
    """Corollary 10.10 (power scheme, average spectral error).

    [(1 + sqrt(k/(p-1))) sigma_{k+1}^{2q+1}
      + e sqrt(k+p)/p (sum_{j>k} sigma_j^{2(2q+1)})^{1/2}]^{1/(2q+1)}
    """
    s = np.asarray(sigma, dtype=np.float64)
    e = 2 * q + 1
    inner = ((1.0 + np.sqrt(k / (p - 1.0))) * s[k] ** e
             + np.e * np.sqrt(k + p) / p * _tail(s, k, power=e))
    return float(inner ** (1.0 / e))
