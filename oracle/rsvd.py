"""The randomized SVD, step by step, in FP64 on the CPU.

TEST INFRASTRUCTURE (see the package docstring): only tests, the smoke check
and the benchmark's CPU-baseline leg use this module.

Each function follows one procedure of the paper in its own order and
notation.  Library primitives stand in for single steps and nothing more:
numpy matrix products, Householder QR and dense SVD (LAPACK), and numpy's FFT.
No blocking, fusion or reordering beyond what the paper states.

The one reading the paper leaves open is which QR produces "an orthonormal
basis for the range of Y" (Section 4.1 allows Gram-Schmidt with double
orthogonalization, Householder or Givens).  The oracle uses Householder QR and
then flips column signs so that R has a positive real diagonal; for a full-rank
Y that Q is unique, and it is the Q every other stable QR (CholeskyQR2 included)
returns in exact arithmetic.
"""

import numpy as np

from . import philox


def qr_pos(Y):
    """Thin QR of Y with diag(R) real and positive.

    Householder QR through LAPACK (numpy.linalg.qr), then each column of Q is
    multiplied by the phase of the matching diagonal entry of R (and that row
    of R by its conjugate), which leaves the product QR unchanged.
    """
    Q, R = np.linalg.qr(Y, mode="reduced")
    d = np.diag(R).copy()
    phase = np.ones_like(d)
    nz = np.abs(d) > 0
    phase[nz] = d[nz] / np.abs(d[nz])
    Q = Q * phase[None, :]
    R = np.conj(phase)[:, None] * R
    return Q, R


def adj(M):
    """Conjugate transpose (the paper's *)."""
    return np.conj(M).T


# ---------------------------------------------------------------------------
# Stage A: range finders (Section 4)
# ---------------------------------------------------------------------------

def gaussian_test_matrix(n, l, seed, stream=0, dtype=np.float64):
    """Algorithm 4.1, step 1: n x l standard Gaussian test matrix.

    Drawn from the counter-based generator in oracle.philox and rounded to the
    working dtype (round-to-nearest-even) exactly as the working-precision path
    stores it; returned in FP64.
    """
    return philox.round_to_dtype(philox.gaussian_omega(n, l, seed, stream), dtype)


def randomized_range_finder(A, Omega):
    """Algorithm 4.1 (Randomized Range Finder), steps 2-3.

    Y = A Omega, then Q = an orthonormal basis of range(Y) from Y = QR.
    """
    Y = A @ Omega
    Q, _ = qr_pos(Y)
    return Q


def randomized_power_iteration(A, Omega, q):
    """Algorithm 4.3 (Randomized Power Iteration).

    Y = (A A*)^q A Omega by alternating applications of A and A*, with no
    orthonormalization in between; then Q from the QR of Y.  Section 4.5 warns
    that rounding destroys small singular directions here; the oracle keeps it
    only to show that Algorithm 4.4 spans the same space in exact arithmetic.
    """
    Y = A @ Omega
    for _ in range(q):
        Y = A @ (adj(A) @ Y)
    Q, _ = qr_pos(Y)
    return Q


def randomized_subspace_iteration(A, Omega, q):
    """Algorithm 4.4 (Randomized Subspace Iteration).

    Y0 = A Omega = Q0 R0; for j = 1..q: Yt_j = A* Q_{j-1} = Qt_j Rt_j and
    Y_j = A Qt_j = Q_j R_j; return Q = Q_q.  A QR follows every application
    of A or A*, 2q + 1 in all.
    """
    Q, _ = qr_pos(A @ Omega)
    for _ in range(q):
        Qt, _ = qr_pos(adj(A) @ Q)
        Q, _ = qr_pos(A @ Qt)
    return Q


def srft_sketch(A, d, R):
    """Algorithm 4.5 (Fast Randomized Range Finder), step 2: Y = A Omega for the SRFT.

    Omega = sqrt(n/l) D F R (Section 4.6) with F the unitary DFT,
    f_pq = n^(-1/2) exp(-2 pi i (p-1)(q-1)/n).  Column t of A Omega is
    sqrt(n/l) n^(-1/2) sum_p A[:, p] d_p exp(-2 pi i p R_t / n), i.e. the
    unnormalized forward DFT of each row of A D, sampled at frequency R_t and
    scaled by 1/sqrt(l).  The full transform is taken and then sampled, the
    variant the remark after Algorithm 4.5 recommends; numpy's forward FFT has
    exactly the exp(-2 pi i k p / n) sign convention.
    """
    n = A.shape[1]
    l = len(R)
    X = np.fft.fft(A * d[None, :], axis=1)
    assert X.shape[1] == n
    return X[:, np.asarray(R)] / np.sqrt(l)


def srft_test_matrix(n, d, R):
    """The n x l SRFT matrix sqrt(n/l) D F R written out entry by entry (Section 4.6).

    Dense and O(n l); used only to pin srft_sketch on small sizes.
    """
    l = len(R)
    p = np.arange(n)[:, None]
    cols = np.asarray(R)[None, :]
    F_cols = np.exp(-2j * np.pi * p * cols / n) / np.sqrt(n)
    return np.sqrt(n / l) * d[:, None] * F_cols


def fast_randomized_range_finder(A, d, R):
    """Algorithm 4.5: SRFT sketch followed by the QR of step 3."""
    Q, _ = qr_pos(srft_sketch(A, d, R))
    return Q


# ---------------------------------------------------------------------------
# The real tailoring of the SRFT.  Section 4.6 notes that the scheme can be
# tailored to the real or the complex case and treats the complex one.  For a
# real A the real tailoring replaces F by the real orthonormal Fourier basis
# F_r = F T, where T is the fixed unitary matrix that mixes each frequency pair
# (q, n - q) into a cosine and a sine column:
#   column 0          : f_0                      = n^-1/2
#   column n/2        : f_{n/2}                  = n^-1/2 (-1)^p
#   column q, q < n/2 : (f_q + f_{n-q}) / sqrt 2 = sqrt(2/n) cos(2 pi p q / n)
#   column q, q > n/2 : with q' = n - q,
#                       i (f_{q'} - f_q) / sqrt 2 = sqrt(2/n) sin(2 pi p q' / n)
# (n even).  Omega = sqrt(n/l) D F_r R stays real, and so do Y, Q, B, U, V.
# ---------------------------------------------------------------------------

def real_fourier_matrix(n):
    """F_r (n x n, real orthogonal) written out entry by entry; n even."""
    if n % 2:
        raise ValueError("the real Fourier basis here needs an even n")
    p = np.arange(n)[:, None]
    q = np.arange(n)[None, :]
    Fr = np.zeros((n, n))
    Fr[:, 0] = 1.0 / np.sqrt(n)
    Fr[:, n // 2] = (-1.0) ** np.arange(n) / np.sqrt(n)
    lo = (q > 0) & (q < n // 2)
    hi = q > n // 2
    Fr += np.where(lo, np.sqrt(2.0 / n) * np.cos(2 * np.pi * p * q / n), 0.0)
    Fr += np.where(hi, np.sqrt(2.0 / n) * np.sin(2 * np.pi * p * (n - q) / n), 0.0)
    return Fr


def real_srft_test_matrix(n, d, R):
    """Omega = sqrt(n/l) D F_r R, dense (for pins on small n)."""
    l = len(R)
    return np.sqrt(n / l) * d[:, None] * real_fourier_matrix(n)[:, np.asarray(R)]


def real_srft_sketch(A, d, R):
    """Y = A Omega for the real SRFT, from one FFT per row (Algorithm 4.5, step 2).

    With X the unnormalized forward DFT of a row of A D, column t of Y is
    sqrt(n/l) times the row's coefficient on column R_t of F_r:
      R_t = 0        : X[0] / sqrt(l)
      R_t = n/2      : X[n/2] / sqrt(l)
      R_t < n/2      : sqrt(2/l) Re X[R_t]
      R_t > n/2      : -sqrt(2/l) Im X[n - R_t]
    """
    n = A.shape[1]
    l = len(R)
    X = np.fft.fft(A * d[None, :], axis=1)
    Y = np.empty((A.shape[0], l))
    for t, q in enumerate(np.asarray(R)):
        if q == 0:
            Y[:, t] = X[:, 0].real / np.sqrt(l)
        elif 2 * q == n:
            Y[:, t] = X[:, n // 2].real / np.sqrt(l)
        elif 2 * q < n:
            Y[:, t] = np.sqrt(2.0 / l) * X[:, q].real
        else:
            Y[:, t] = -np.sqrt(2.0 / l) * X[:, n - q].imag
    return Y


# ---------------------------------------------------------------------------
# Stage B: Direct SVD (Section 5.1)
# ---------------------------------------------------------------------------

def direct_svd(A, Q):
    """Algorithm 5.1 (Direct SVD): B = Q* A; B = Ut S V*; U = Q Ut.

    The SVD of the small matrix is LAPACK's (numpy.linalg.svd), singular values
    descending.  Returns (U, S, V, B) with V = (V*)* so that A ~ U diag(S) V*.
    """
    B = adj(Q) @ A
    Ut, S, Vh = np.linalg.svd(B, full_matrices=False)
    U = Q @ Ut
    return U, S, adj(Vh), B


def truncate(U, S, V, k):
    """Keep the k dominant singular triplets (the truncation remark in Section 5.1)."""
    return U[:, :k], S[:k], V[:, :k]


def normalize_signs(U, V):
    """Fix the sign (phase) freedom of singular vector pairs.

    Singular vectors are unique only up to a common unit scalar per pair.  For
    each j the pair (u_j, v_j) is multiplied by the conjugate phase of the
    largest-magnitude entry of v_j (lowest index on ties), which makes that
    entry real and positive.
    """
    U = np.array(U, copy=True)
    V = np.array(V, copy=True)
    for j in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, j])))
        a = V[i, j]
        if a == 0:
            continue
        ph = np.conj(a / np.abs(a))
        V[:, j] *= ph
        U[:, j] *= ph
    return U, V


def rsvd(A, k, p, q=0, *, seed=0, stream=0, sketch="gaussian", dtype=np.float64,
         Omega=None):
    """Randomized SVD: Stage A then Stage B (Section 1.6 prototype, l = k + p).

    Stage A is Algorithm 4.4 for the Gaussian sketch (it reduces to Algorithm
    4.1 at q = 0) or Algorithm 4.5 for the SRFT (q = 0 only: Section 4.6 notes
    that the structured sketch does not speed up the power scheme) -- "srft"
    is the real tailoring (real Fourier basis, real Y), "srft_complex" the
    complex case the paper writes out.  Stage B is Algorithm 5.1 followed by
    truncation to rank k.

    A must already hold exactly the values the working-precision path reads
    (an FP32 matrix promoted to FP64).  The Gaussian Omega is drawn by
    oracle.philox and rounded to `dtype`; pass Omega to override it.
    Returns a dict with the test matrix, Q, B and the full and truncated
    factors.
    """
    A = np.asarray(A)
    m, n = A.shape
    l = k + p
    if not (1 <= k and p >= 0 and l <= min(m, n) and q >= 0):
        raise ValueError("need 1 <= k, p >= 0, k + p <= min(m, n), q >= 0")
    out = {}
    if sketch == "gaussian":
        if Omega is None:
            Omega = gaussian_test_matrix(n, l, seed, stream, dtype)
        out["Omega"] = Omega
        Q = randomized_subspace_iteration(A, Omega, q)
    elif sketch in ("srft", "srft_complex"):
        if q != 0:
            raise ValueError("the SRFT range finder is used with q = 0")
        d = philox.srft_signs(n, seed, stream)
        R = philox.srft_sample(n, l, seed, stream)
        out["d"], out["R"] = d, R
        if sketch == "srft":   # real tailoring (real A): Y real
            Q, _ = qr_pos(real_srft_sketch(A, d, R))
        else:                  # complex case of Section 4.6
            Q = fast_randomized_range_finder(A, d, R)
    else:
        raise ValueError("sketch must be 'gaussian', 'srft' or 'srft_complex'")
    U, S, V, B = direct_svd(A, Q)
    Uk, Sk, Vk = truncate(U, S, V, k)
    out.update(Q=Q, B=B, U=U, S=S, V=V, Uk=Uk, Sk=Sk, Vk=Vk)
    return out
