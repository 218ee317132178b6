"""The fixed-precision range finder (Section 4.3-4.4), in FP64 on the CPU.

TEST INFRASTRUCTURE (see the package docstring): only tests, the smoke check
and the benchmark's CPU-baseline leg use this module.

Given A, a tolerance eps and an integer r, the range finder grows an
orthonormal basis Q until ||(I - Q Q*) A|| <= eps holds with high probability.
The test is the a posteriori estimate of eq. (4.3), from the lemma after it:
for r independent standard Gaussian vectors w_i,
    ||B|| <= 10 sqrt(2/pi) max_i ||B w_i||   except with probability 10^-r,
applied to B = (I - Q Q*) A, whose products B w_i are exactly the projected
samples the basis is grown from.

Two organizations of the same method:
  * adaptive_range_finder: Algorithm 4.2 as stated, one sample at a time, with
    the window of the r most recent projected samples as the test;
  * blocked_adaptive_range_finder: the samples taken a block at a time (the
    remark after Algorithm 4.2), the guess for the rank doubled at each step
    (Section 4.3: "start with 32 samples, compute another 32, then another 64"):
    block t is first used as the test of the current basis; if it fails, its
    range is appended.  This is what the GPU runs, on the same test matrix.
Library primitives stand in for single steps only: numpy products and norms,
and Householder QR (LAPACK) for the orthonormalization of a block.
"""

import numpy as np

from .rsvd import qr_pos


def errorest_factor():
    """10 sqrt(2/pi): the multiplier of eq. (4.3) (alpha = 10 in the lemma)."""
    return 10.0 * np.sqrt(2.0 / np.pi)


def posterior_estimate(B, W):
    """The right-hand side of eq. (4.3) for B and the Gaussian vectors in the columns of W:
    10 sqrt(2/pi) max_i ||B w_i||."""
    return errorest_factor() * float(np.max(np.linalg.norm(B @ W, axis=0)))


def adaptive_range_finder(A, eps, r, Omega):
    """Algorithm 4.2 (Adaptive Randomized Range Finder), step by step.

    Omega's columns are the Gaussian vectors w^(1), w^(2), ... in the order the
    algorithm draws them (steps 1 and 10).  Returns (Q, j): the m x j basis.
    The loop also stops when j reaches min(m, n) or the columns of Omega run
    out (the algorithm is then past the point where its test can be applied).
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    thresh = eps / errorest_factor()
    jmax = min(m, n, Omega.shape[1] - r)
    y = {i: A @ Omega[:, i - 1] for i in range(1, r + 1)}        # steps 1-2
    j = 0                                                         # step 3
    Q = np.zeros((m, 0))                                          # step 4
    while max(np.linalg.norm(y[j + i]) for i in range(1, r + 1)) > thresh and j < jmax:  # step 5
        j += 1                                                    # step 6
        y[j] = y[j] - Q @ (Q.T @ y[j])                            # step 7
        q = y[j] / np.linalg.norm(y[j])                           # step 8
        Q = np.column_stack([Q, q])                               # step 9
        w = Omega[:, j + r - 1]                                   # step 10
        y[j + r] = A @ w - Q @ (Q.T @ (A @ w))                    # step 11
        for i in range(j + 1, j + r):                             # steps 12-14
            y[i] = y[i] - q * (q @ y[i])
    return Q, j


def block_schedule(b0, lmax):
    """Block sizes of the blocked range finder: b0, b0, 2 b0, 4 b0, ... until the basis holds
    lmax = b0 2^T columns, then the final test block takes r columns (see below)."""
    sizes, cols = [], 0
    while cols < lmax:
        b = b0 if cols == 0 else cols
        sizes.append(b)
        cols += b
    return sizes


def blocked_adaptive_range_finder(A, eps, r, b0, lmax, Omega):
    """Algorithm 4.2 with the samples taken in blocks of doubling size.

    Omega (n x (lmax + r)) holds the test vectors in the order they are used.
    For block t (columns c .. c + b_t of Omega): Y = A Omega_t, projected onto
    range(Q)-perp twice (the reprojection of steps 7-8, for the whole block);
    its columns are (I - Q Q*) A w for fresh Gaussian w, so if all b_t >= r of
    them have norm <= eps / (10 sqrt(2/pi)), Q passes the test of eq. (4.3) and
    is returned.  Otherwise Q <- [Q, Q_b] with Q_b the orthonormal factor of Y,
    projected once more and refactored (block Gram-Schmidt with
    reorthogonalization).  When Q holds lmax columns, one last block of r
    fresh columns gives the final estimate.

    Returns dict(Q, l, est, converged, tested): est is the estimate of eq. (4.3)
    from the last block tested (an upper bound on ||(I - Q Q*) A|| with
    probability at least 1 - 10^-b), converged whether it is <= eps.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if b0 < r or lmax % b0 != 0 or (lmax // b0) & (lmax // b0 - 1):
        raise ValueError("need b0 >= r and lmax = b0 * 2^T")
    Q = np.zeros((m, 0))
    c = 0
    tested = []
    for b in block_schedule(b0, lmax) + [r]:
        Y = A @ Omega[:, c:c + b]
        c += b
        for _ in range(2):
            Y = Y - Q @ (Q.T @ Y)
        est = errorest_factor() * float(np.max(np.linalg.norm(Y, axis=0)))
        tested.append(est)
        if est <= eps or Q.shape[1] == lmax:
            return dict(Q=Q, l=Q.shape[1], est=est, converged=est <= eps, tested=tested)
        # the block's orthonormal basis, made orthogonal to Q once more: when Y has columns at
        # roundoff level (the basis already holds most of range(A)), their normalized directions
        # are arbitrary and carry components along Q, which a second projection removes
        Qb, _ = qr_pos(Y)
        for _ in range(2):
            Qb = Qb - Q @ (Q.T @ Qb)
        Qb, _ = qr_pos(Qb)
        Q = np.column_stack([Q, Qb])
    raise AssertionError("unreachable: the schedule ends with the final test block")
