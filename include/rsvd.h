/*
 * rsvd.h -- C ABI of the MI355X (gfx950) randomized SVD library (librsvd.so).
 *
 * The library computes the two-stage randomized SVD of Halko, Martinsson and
 * Tropp, "Finding structure with randomness" (SIAM Review 2011):
 *
 *   Stage A (range finding): draw a test matrix Omega, form Y = (A A*)^q A Omega
 *     with an orthonormalization after every application of A or A*
 *     (Algorithm 4.4, randomized subspace iteration; Algorithm 4.1 when q = 0),
 *     or, for the SRFT test matrix of Section 4.6, Y = A Omega by FFT
 *     (Algorithm 4.5).  Q is an orthonormal basis of range(Y).  A is real, and
 *     the SRFT is its real tailoring (Section 4.6 notes that the transform can
 *     be set up for the real or the complex case): F is replaced by the real
 *     orthonormal Fourier basis F_r, whose columns are the constant, the
 *     alternating and, for 0 < q < n/2, sqrt(2) cos(2 pi p q / n) and
 *     sqrt(2) sin(2 pi p q / n), each over sqrt(n).  Every output stays real.
 *   Stage B (Algorithm 5.1, direct SVD): B = Q* A, an SVD of the small matrix
 *     B = U~ S V*, U = Q U~, then truncation to the k leading triplets (the
 *     truncation remark of Section 5.1).
 *
 * The problem statement follows the fixed-rank problem of Section 1.3: an
 * m x n matrix A, the rank k sought, p extra samples (l = k + p columns in
 * the test matrix), and q power steps (Section 1.6, Section 4.5).
 *
 * Conventions for every call
 * --------------------------
 *  * All matrices are row-major.  A has leading dimension lda >= n (elements).
 *    Every other matrix is dense with leading dimension equal to its column
 *    count.
 *  * Element type: float (RSVD_F32) or double (RSVD_F64), chosen by
 *    problem->dtype, for A, Omega, Q, Bt, U, S and V (all real, with either
 *    sketch).
 *  * Pointers named A, Q, Bt, U, S, V, Omega and ws are DEVICE pointers on the
 *    handle's device.  The problem descriptor is a HOST pointer.  `stream` is
 *    a hipStream_t (NULL = the default stream) on which every kernel of the
 *    call is enqueued; calls return without synchronizing.
 *  * Ownership: the caller owns every buffer.  The library never allocates or
 *    frees memory in these calls (the batched calls excepted: the first call
 *    for a new batch allocates the batch's launch tables, owned by the
 *    handle);
 *    scratch space is the caller's workspace `ws` of at least
 *    rsvd_workspace_bytes(problem) bytes, 256-byte aligned.  Its
 *    contents are undefined between calls (except as noted for rsvd_project ->
 *    rsvd_svd, which carry nothing through it).
 *  * Errors: argument errors are detected on the host before any launch and
 *    returned synchronously (RSVD_E_INVAL, RSVD_E_WORKSPACE,
 *    RSVD_E_UNSUPPORTED); a HIP launch error returns RSVD_E_DEVICE.  Numerical
 *    conditions found on the device (a Cholesky pivot that needed a shift, a
 *    non-finite value, a Jacobi sweep cap) are recorded in the handle's device
 *    status word and read by rsvd_device_status.  No call throws.
 *  * A handle is not thread-safe; calls that share a handle must be ordered.
 */
#ifndef RSVD_H
#define RSVD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rsvd_status {
  RSVD_OK = 0,
  RSVD_E_INVAL = 1,        /* bad argument: null pointer, shape or parameter out of range */
  RSVD_E_WORKSPACE = 2,    /* workspace null or smaller than rsvd_workspace_bytes() */
  RSVD_E_DEVICE = 3,       /* a HIP call or kernel launch failed */
  RSVD_E_UNSUPPORTED = 4,  /* valid problem outside what the library implements */
  RSVD_E_BREAKDOWN = 5,    /* device status: a Cholesky pivot was not positive (a shift was applied) */
  RSVD_E_NONFINITE = 6,    /* device status: a NaN or Inf reached a Gram matrix */
  RSVD_E_NOCONV = 7        /* device status: Jacobi SVD hit its sweep cap */
} rsvd_status;

/* problem->dtype */
enum { RSVD_F32 = 0, RSVD_F64 = 1 };
/* problem->sketch: the test matrix of Stage A */
enum {
  RSVD_GAUSSIAN = 0,  /* i.i.d. N(0,1) n x l (Section 4.1) */
  RSVD_SRFT = 1,      /* sqrt(n/l) D F_r R with D = random +-1 signs and F_r the real
                         orthonormal Fourier basis (Section 4.6); q must be 0 */
  RSVD_GSRFT = 2      /* D'' Theta' D' Theta (sqrt(n/l) D F_r R): the SRFT behind two chains
                         of random Givens rotations, each a random permutation followed by
                         rotations in the planes (j, j + 1) with angles uniform on [0, 2 pi),
                         and random +-1 diagonals D', D'' (the remark on random Givens
                         rotations in Section 4.6, real form).  q must be 0; n a power of
                         two, 8 <= n <= 16384 (FP32) or 8192 (FP64).  The workspace holds a
                         transformed copy of A (m x n elements) */
};
/* problem->prec: arithmetic of the products that stream A (the sketch,
 * power-step and projection GEMMs).  Gram matrices, Cholesky factors and the
 * small SVD are always FP64. */
enum {
  RSVD_NATIVE = 0,  /* products in the element type on FP32 / FP64 MFMA */
  RSVD_BF16 = 1,    /* FP32 data rounded to bfloat16, one BF16 MFMA product, FP32 accumulation */
  RSVD_BF16X3 = 2   /* split-precision: a = a_hi + a_lo (bfloat16 each), three BF16 MFMA
                       products a_hi b_hi + a_hi b_lo + a_lo b_hi, FP32 accumulation */
};

/* Device status bits (rsvd_device_status) */
enum {
  RSVD_FLAG_SHIFTED = 1,    /* a Cholesky factorization needed a diagonal shift */
  RSVD_FLAG_NONFINITE = 2,  /* a Gram matrix held NaN/Inf */
  RSVD_FLAG_NOCONV = 4      /* the Jacobi SVD stopped at its sweep cap */
};

typedef struct rsvd_problem {
  int64_t m, n;     /* A is m x n */
  int64_t lda;      /* leading dimension of A in elements, lda >= n */
  int32_t k;        /* target rank, 1 <= k */
  int32_t p;        /* oversampling, p >= 0; l = k + p <= min(m, n) and l <= RSVD_MAX_L */
  int32_t q;        /* power steps, q >= 0 (must be 0 with the SRFT sketch) */
  int32_t dtype;    /* RSVD_F32 or RSVD_F64 */
  int32_t sketch;   /* RSVD_GAUSSIAN, RSVD_SRFT or RSVD_GSRFT */
  int32_t prec;     /* RSVD_NATIVE, RSVD_BF16 or RSVD_BF16X3 (the last two need RSVD_F32) */
  uint64_t seed;    /* Philox4x64-10 key word 0 */
  uint64_t stream_id; /* Philox counter word 1: independent draws for the same seed */
} rsvd_problem;

/* Largest number of samples l = k + p the library supports (one workgroup
 * holds the l x l factors of the small FP64 steps in its local memory). */
#define RSVD_MAX_L 128

typedef struct rsvd_handle_s* rsvd_handle;

/* Create a handle on HIP device `device`: records the device and allocates the
 * handle's 16-byte device status word.  The only allocation the library makes. */
rsvd_status rsvd_create(rsvd_handle* handle, int device);
rsvd_status rsvd_destroy(rsvd_handle handle);

/* Pure host checks of a problem descriptor (no device, no handle).  RSVD_OK,
 * RSVD_E_INVAL (violates the problem statement: k < 1, p < 0, q < 0,
 * l > min(m, n), lda < n, unknown enum) or RSVD_E_UNSUPPORTED (l > RSVD_MAX_L,
 * BF16 precisions with FP64 data; with the SRFT: q > 0, n not a power of two,
 * n < 8, or n above 16384 (FP32) / 8192 (FP64), the largest row one
 * workgroup transforms in its local memory). */
rsvd_status rsvd_validate(const rsvd_problem* problem);

/* Bytes of workspace every call below needs for `problem` (0 if invalid).
 * One size serves all four hot-path calls. */
size_t rsvd_workspace_bytes(const rsvd_problem* problem);

const char* rsvd_status_string(rsvd_status status);

/* --- The hot path ------------------------------------------------------- */

/* Stage A, first application: Algorithm 4.1 (Gaussian; step 2 of Algorithm
 * 4.4) or Algorithm 4.5 (SRFT).  Draws Omega from (seed, stream_id), forms
 * Y = A Omega and writes a basis Q (m x l) of range(Y).  With problem->q == 0
 * Q is orthonormal, computed by CholeskyQR2 (two passes of Gram -> Cholesky ->
 * Y R^-1, FP64 Gram and Cholesky, a shifted third pass when needed).  With
 * q > 0 the power steps of rsvd_power_iter follow and Q only feeds the first
 * of them: one CholeskyQR pass (all three when the first needed a shift), a
 * well-conditioned basis orthonormal to about u kappa(Y) (see
 * rsvd_power_iter).  A: m x n (lda); Q: m x l output.  With the SRFT, Y is formed in
 * the element type by one length-n real FFT per row of A D (the full
 * transform, then the l sampled frequencies: the variant the remark after
 * Algorithm 4.5 recommends); problem->prec does not apply to it. */
rsvd_status rsvd_range_finder(rsvd_handle handle, const rsvd_problem* problem,
                              const void* A, void* Q, void* ws, size_t ws_bytes,
                              hipStream_t stream);

/* Stage A, power steps: Algorithm 4.4 steps 3-6.  For j = 1..q:
 * Qt = orth(A* Q), Q = orth(A Qt).  The last Q is orthonormalized by
 * CholeskyQR2 (FP64 Gram and Cholesky, a shifted third pass when needed).
 * The bases before it only feed the next product and take one CholeskyQR
 * pass (all three when the first needed a shift): they are
 * orthonormal to about u kappa (u the element type's unit roundoff, kappa
 * the condition number of the product), a well-conditioned basis of the
 * same range.  Q (m x l) is read and overwritten in place; its input need
 * only be a well-conditioned basis.  A no-op when q = 0. */
rsvd_status rsvd_power_iter(rsvd_handle handle, const rsvd_problem* problem,
                            const void* A, void* Q, void* ws, size_t ws_bytes,
                            hipStream_t stream);

/* Stage B, step 1 of Algorithm 5.1: B = Q* A.  Written as its transpose
 * Bt = A^T conj(Q) (n x l, row-major), i.e. B stored column-major: Bt[j*l + i]
 * = B[i][j]. */
rsvd_status rsvd_project(rsvd_handle handle, const rsvd_problem* problem,
                         const void* A, const void* Q, void* Bt, void* ws,
                         size_t ws_bytes, hipStream_t stream);

/* Stage B, steps 2-3 of Algorithm 5.1 plus truncation to rank k: an SVD of the
 * small matrix B = U~ S V* in FP64, U = Q U~, and the k leading triplets.  For
 * FP64 data: CholeskyQR of B* = Q_B R, one-sided Jacobi on R^T (backward
 * stable); for FP32 data: the eigendecomposition of the Gram B B* = U~ S^2 U~*
 * (Householder tridiagonalization, bisection, inverse iteration).  Bt: n x l (from rsvd_project);
 * Q: m x l; outputs U: m x k, S: k (real, descending), V: n x k, with
 * A ~ U diag(S) V*. */
rsvd_status rsvd_svd(rsvd_handle handle, const rsvd_problem* problem,
                     const void* Bt, const void* Q, void* U, void* S, void* V,
                     void* ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes of rsvd_full (0 if the problem is invalid): Q and Bt as well
 * as the hot-path workspace. */
size_t rsvd_full_workspace_bytes(const rsvd_problem* problem);

/* rsvd_range_finder, rsvd_power_iter, rsvd_project and rsvd_svd in one call,
 * with Q and Bt kept in `ws`: U, S, V as rsvd_svd writes them, bit for bit the
 * four calls' results.  The first call for given (problem, A, U, S, V, ws)
 * captures the launches in a HIP graph owned by the handle (kept with the
 * batched plans, eight at most, freed by rsvd_destroy); later calls with the
 * same arguments replay it, so a small problem pays no host work per kernel.
 * The graph reads and writes the same buffers on every replay: new contents of
 * A are decomposed, and calls that overlap on one workspace race. */
rsvd_status rsvd_full(rsvd_handle handle, const rsvd_problem* problem, const void* A,
                      void* U, void* S, void* V, void* ws, size_t ws_bytes, hipStream_t stream);

/* --- Fixed-precision range finder ---------------------------------------- */

/* Workspace bytes of rsvd_range_finder_tol (0 if the problem or r is not
 * accepted, see below). */
size_t rsvd_range_finder_tol_workspace_bytes(const rsvd_problem* problem, int32_t r);

/* The fixed-precision problem of Section 1.3: an orthonormal Q (m x l) with
 * ||(I - Q Q*) A|| <= eps, l found by the method.  Algorithm 4.2 (Adaptive
 * Randomized Range Finder) with its samples taken in blocks (the remark after
 * Algorithm 4.2) whose sizes double the guess for the rank (Section 4.3):
 * b0, b0, 2 b0, 4 b0, ... with b0 = problem->k, up to the capacity
 * lmax = problem->k + problem->p, which must be b0 times a power of two
 * (l is then one of 0, b0, 2 b0, 4 b0, ..., lmax).  Each block first tests the
 * current basis by the a posteriori estimate of eq. (4.3):
 *   est = 10 sqrt(2/pi) max_i ||(I - Q Q*) A w_i||
 * over its b >= r fresh Gaussian vectors w_i (the bound ||(I - Q Q*) A|| <= est
 * holds with probability at least 1 - 10^-b); if est <= eps the call returns Q,
 * otherwise the block's samples, projected twice onto range(Q)-perp and
 * orthonormalized (CholeskyQR2; projected and refactored once more), are
 * appended.  When Q holds lmax columns a last block of r vectors gives the
 * final estimate.  The vectors w come from one n x (lmax + r) Gaussian test
 * matrix drawn from (seed, stream_id) by the generator contract of
 * rsvd_draw_omega, columns used in order.  problem->prec sets the arithmetic
 * of the products with A; q must be 0 and the sketch Gaussian
 * (RSVD_E_UNSUPPORTED otherwise); 1 <= r <= k (RSVD_E_INVAL otherwise).
 * Q: m x lmax DEVICE buffer (row-major, leading dimension lmax), of which the
 * first *l_out columns are written.  *l_out and *est_out are HOST outputs; the
 * call synchronizes `stream` after every block (the host takes the decision).
 * est > eps on return means the capacity was reached first. */
rsvd_status rsvd_range_finder_tol(rsvd_handle handle, const rsvd_problem* problem, double eps, int32_t r,
                                  const void* A, void* Q, int32_t* l_out, double* est_out, void* ws,
                                  size_t ws_bytes, hipStream_t stream);

/* --- Stage B for symmetric and positive semidefinite A ------------------- */

/* Both calls take the problem with m == n (A is n x n, row-major, leading
 * dimension lda) and a basis Q (n x l, l = k + p, row-major with leading
 * dimension l, orthonormal columns: the output of rsvd_range_finder or
 * rsvd_power_iter); problem->prec sets the arithmetic of the product A Q, the
 * only pass over A; q, sketch, seed and stream_id are not used.  Workspace:
 * rsvd_workspace_bytes(problem).  Outputs, DEVICE buffers in the element type:
 * U (n x k, row-major, leading dimension k) and Lam (k).  Errors as for the
 * hot-path calls; m != n is RSVD_E_INVAL.
 *
 * rsvd_eigh: Algorithm 5.3 (direct eigenvalue decomposition, Section 5.3) for
 * symmetric A: B = Q^T A Q (l x l, replaced by its symmetric part), its
 * eigendecomposition B = V Lambda V^T, U = Q V.  The k eigenpairs of largest
 * |lambda| are kept, in decreasing order of |lambda| (equal magnitudes: the
 * positive one first); Lam holds the signed eigenvalues.  With k = l,
 * ||A - U Lam U^T|| <= 2 ||A - Q Q^T A|| (Section 5.3).
 *
 * rsvd_nystrom: Algorithm 5.5 (eigenvalue decomposition via the Nystrom
 * method, Section 5.4) for positive semidefinite A: B1 = A Q, B2 = Q^T B1 (its
 * symmetric part) = C^T C (Cholesky, C upper triangular), F = B1 C^-1,
 * F = U Sigma V^T, Lam = Sigma^2 (the k largest, decreasing).  B2 must be
 * positive definite to working precision (the l-th eigenvalue of A above the
 * rounding of the product A Q, about sqrt(n) u ||A|| for element precision u):
 * otherwise the Cholesky factorization is restarted on B2 + s I with the
 * shifted-CholeskyQR shift and RSVD_FLAG_SHIFTED is raised in the device
 * status word, and the result is that of the shifted core. */
rsvd_status rsvd_eigh(rsvd_handle handle, const rsvd_problem* problem, const void* A, const void* Q, void* U,
                      void* Lam, void* ws, size_t ws_bytes, hipStream_t stream);
rsvd_status rsvd_nystrom(rsvd_handle handle, const rsvd_problem* problem, const void* A, const void* Q, void* U,
                         void* Lam, void* ws, size_t ws_bytes, hipStream_t stream);

/* rsvd_eigh_onepass: Algorithm 5.6 (eigenvalue decomposition in one pass,
 * Section 5.5) for symmetric A (m == n, n x n, row-major, leading dimension
 * lda): A is read once, by the sample Y = A Omega with Omega (n x l, l = k + p)
 * drawn from (seed, stream_id) exactly as rsvd_draw_omega draws it.  Q is the
 * n x k matrix of the k leading left singular vectors of Y when p > 0 (the
 * oversampling of the remark that closes Section 5.5) and an orthonormal basis
 * of range(Y) when p == 0; B (k x k) is the symmetric part of the standard
 * least-squares solution of B (Q^T Omega) = Q^T Y (Q^T Omega has full row
 * rank); B = V Lambda V^T; U = Q V.  Outputs, DEVICE buffers in the element
 * type: U (n x k, leading dimension k) and Lam (k), all k pairs in decreasing
 * |lambda| (equal magnitudes: the positive one first).  Workspace:
 * rsvd_workspace_bytes(problem).  The Gaussian sketch only
 * (RSVD_E_UNSUPPORTED otherwise); q is not used; m != n is RSVD_E_INVAL. */
rsvd_status rsvd_eigh_onepass(rsvd_handle handle, const rsvd_problem* problem, const void* A, void* U, void* Lam,
                              void* ws, size_t ws_bytes, hipStream_t stream);

/* rsvd_svd_onepass: the single-pass factorization of a general A that
 * Section 5.5 describes after Algorithm 5.6.  Omega (n x l, l = k + p) is drawn from (seed, stream_id) as
 * rsvd_draw_omega draws it and Omegat (m x l) from (seed, stream_id with its
 * top bit flipped); Y = A Omega and Yt = A^T Omegat are the only products with
 * A (two launches here, each reading A once: with A resident in device memory
 * a fused launch would trade the second read for partial sums of the same
 * size); Q, Qt = CholeskyQR2 bases of their ranges (Q^T Y = R, Qt^T Yt = Rt);
 * B (l x l) = the minimum-residual solution of B (Qt^T Omega) = R and
 * B^T (Q^T Omegat) = Rt, through its normal equations B G1 + G2 B = C and the
 * eigendecompositions of G1 = M1 M1^T and G2 = M2 M2^T; B = Ub S Vb^T;
 * U = Q Ub_k, V = Qt Vb_k.  Outputs and workspace as rsvd_full's hot-path
 * calls: U (m x k), S (k, descending), V (n x k), DEVICE buffers in the element
 * type, workspace rsvd_workspace_bytes(problem).  The Gaussian sketch only
 * (RSVD_E_UNSUPPORTED otherwise); q is not used. */
rsvd_status rsvd_svd_onepass(rsvd_handle handle, const rsvd_problem* problem, const void* A, void* U, void* S,
                             void* V, void* ws, size_t ws_bytes, hipStream_t stream);

/* Size of the device array that rsvd_full_static uses as its workspace. */
#define RSVD_STATIC_SCRATCH_BYTES ((size_t)32 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rsvd_full
 * with no workspace argument and no allocation of any kind.  Q, Bt and the
 * hot-path workspace live in a file-scope device array of
 * RSVD_STATIC_SCRATCH_BYTES (32 MiB), one copy per device, held from the
 * library's first use on that device until the process ends; rsvd_create
 * looks up its device address.  The kernels are launched directly on `stream`
 * (no graph), so U, S, V are bit for bit those of rsvd_full and of the four
 * hot-path calls.  A problem whose rsvd_full_workspace_bytes exceeds
 * RSVD_STATIC_SCRATCH_BYTES returns RSVD_E_WORKSPACE before any launch.
 * Every call on one device shares that device's array and leaves its
 * contents behind (nothing in it has to start at zero): calls that overlap on
 * one device -- on different streams, or through different handles -- race. */
rsvd_status rsvd_full_static(rsvd_handle handle, const rsvd_problem* problem, const void* A,
                             void* U, void* S, void* V, hipStream_t stream);

/* --- Differentiation ---------------------------------------------------- */

/* Workspace bytes of rsvd_backward (0 if the problem is invalid or uses the
 * SRFT sketch). */
size_t rsvd_backward_workspace_bytes(const rsvd_problem* problem);

/* Adjoint (vector-Jacobian product) of the map A -> (U, S, V) computed by
 * rsvd_range_finder, rsvd_power_iter, rsvd_project and rsvd_svd for the same
 * problem, with the test matrix held fixed (same seed and stream_id; Gaussian
 * sketch only).  Given the adjoints gU (m x k), gS (k) and gV (n x k) of the
 * outputs (DEVICE, element type, dense row-major), writes gA (m x n, dense
 * row-major, leading dimension n) = sum of gU . dU + gS . dS + gV . dV over a
 * perturbation dA.  The forward is recomputed inside (nothing is kept from an
 * earlier call), then each step is differentiated in reverse: the SVD of the
 * small matrix B (standard thin-SVD derivative, FP64), B = Q* A, every
 * CholeskyQR of the power scheme (gY = (gQ + Q sym(-gQ^T Q)) R^-T, FP64 for
 * the l x l parts) and the products with A; gA is the sum of 2q + 2 rank-l
 * terms, formed by one product.  The derivative exists where B has full rank
 * l, its k leading singular values are distinct and sigma_k > sigma_(k+1);
 * near those points it grows like 1 / (sigma_i^2 - sigma_j^2). */
rsvd_status rsvd_backward(rsvd_handle handle, const rsvd_problem* problem,
                          const void* A, const void* gU, const void* gS,
                          const void* gV, void* gA, void* ws, size_t ws_bytes,
                          hipStream_t stream);

/* The forward of rsvd_backward kept for it: the whole randomized SVD of A
 * (outputs U, S, V as rsvd_svd) computed in an adjoint workspace `ws`
 * (rsvd_backward_workspace_bytes bytes), where it leaves every basis of the
 * power scheme with its triangular factor, B* and the SVD of B.  Every basis
 * is orthonormalized by CholeskyQR2 (the adjoint differentiates exact QR
 * factors), so U, S, V equal the four hot-path calls' (which take one pass for
 * the bases inside the power scheme) up to the element type's rounding.  rsvd_backward_kept then skips the
 * recomputation; the state stays valid while `ws` is not otherwise used. */
rsvd_status rsvd_forward_kept(rsvd_handle handle, const rsvd_problem* problem,
                              const void* A, void* U, void* S, void* V,
                              void* ws, size_t ws_bytes, hipStream_t stream);

/* rsvd_backward from the state rsvd_forward_kept left in `ws` for the same
 * problem and the same contents of A: the adjoint only, gA bit for bit equal to
 * rsvd_backward's.  The state is only read, so the call may be repeated. */
rsvd_status rsvd_backward_kept(rsvd_handle handle, const rsvd_problem* problem,
                               const void* A, const void* gU, const void* gS,
                               const void* gV, void* gA, void* ws, size_t ws_bytes,
                               hipStream_t stream);

/* --- Many independent problems --------------------------------------- */

/* Workspace bytes rsvd_batched needs for `count` problems (0 if any problem is
 * invalid or the batch is not supported). */
size_t rsvd_batched_workspace_bytes(int32_t count, const rsvd_problem* problems);

/* The whole randomized SVD (rsvd_range_finder, rsvd_power_iter, rsvd_project
 * and rsvd_svd in sequence) of `count` independent matrices of different
 * sizes.  problems[i] (HOST array) describes A[i]; every problem must share
 * dtype, prec and q and use the Gaussian sketch (else RSVD_E_INVAL /
 * RSVD_E_UNSUPPORTED); m, n, lda, k, p, seed and stream_id are per problem.
 * A, U, S, V are HOST arrays of `count` DEVICE pointers: A[i] is m x n (lda),
 * U[i] m x k, S[i] k, V[i] n x k, with the layouts of rsvd_svd.  Each step of
 * the sequence is one launch over all problems (the products stream A without
 * a split of K), so the batch fills the GPU where a single small problem
 * cannot.  The first call for given (problems, ws) records the launch
 * sequence, uploads its parameter tables to device memory owned by the handle
 * and captures the launches in a HIP graph; later calls with the same problems
 * and workspace replay the graph.  When only the buffers A, U, S, V differ from
 * the previous call, the sequence is recorded again on the host and its
 * parameter tables are uploaded on `stream` (from pinned host memory owned by
 * the handle) before the replay.  The handle keeps the eight most recent
 * batches, freed by rsvd_destroy.  Results are those of the single-problem
 * calls up to the rounding of the K reduction order. */
rsvd_status rsvd_batched(rsvd_handle handle, int32_t count, const rsvd_problem* problems,
                         const void* const* A, void* const* U, void* const* S,
                         void* const* V, void* ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes rsvd_backward_batched needs for `count` problems (0 if any
 * problem is invalid, uses the SRFT sketch, or the batch is not supported). */
size_t rsvd_backward_batched_workspace_bytes(int32_t count, const rsvd_problem* problems);

/* rsvd_backward for `count` independent problems (the adjoint of rsvd_batched
 * with the same problems): problems[i] (HOST array) as for rsvd_batched, and
 * A, gU, gS, gV, gA HOST arrays of `count` DEVICE pointers with the layouts
 * of rsvd_backward (gA[i] is m x n, leading dimension n).  Each step of the
 * recomputed forward and of the adjoint is one launch over all problems,
 * replayed from a HIP graph as for rsvd_batched (same plan cache, same
 * re-pointing when only the buffers moved).  gA[i] equals rsvd_backward's
 * for problem i up to the rounding of the K reduction order. */
rsvd_status rsvd_backward_batched(rsvd_handle handle, int32_t count, const rsvd_problem* problems,
                                  const void* const* A, const void* const* gU, const void* const* gS,
                                  const void* const* gV, void* const* gA, void* ws, size_t ws_bytes,
                                  hipStream_t stream);

/* rsvd_forward_kept and rsvd_backward_kept for a batch: rsvd_batched_kept is
 * rsvd_batched computed in a workspace of rsvd_backward_batched_workspace_bytes
 * bytes, where it keeps each problem's forward state; rsvd_backward_batched_kept
 * is rsvd_backward_batched from that state (same problems, same contents of
 * every A).  Both replay recorded graphs as rsvd_batched does. */
rsvd_status rsvd_batched_kept(rsvd_handle handle, int32_t count, const rsvd_problem* problems,
                              const void* const* A, void* const* U, void* const* S,
                              void* const* V, void* ws, size_t ws_bytes, hipStream_t stream);
rsvd_status rsvd_backward_batched_kept(rsvd_handle handle, int32_t count, const rsvd_problem* problems,
                                       const void* const* A, const void* const* gU,
                                       const void* const* gS, const void* const* gV,
                                       void* const* gA, void* ws, size_t ws_bytes,
                                       hipStream_t stream);

/* --- Diagnostics ------------------------------------------------------- */

/* The sketch of Stage A on its own: Y = A Omega (m x l, element type of
 * problem->dtype, row-major) with the test matrix the range finder draws --
 * step 2 of Algorithm 4.1 (Gaussian, arithmetic problem->prec) or of
 * Algorithm 4.5 (SRFT, one real FFT per row of A D, element type) -- without
 * the orthonormalization.  Same workspace as the hot-path calls.  For parity
 * tests of the sketch element by element. */
rsvd_status rsvd_sketch(rsvd_handle handle, const rsvd_problem* problem,
                        const void* A, void* Y, void* ws, size_t ws_bytes,
                        hipStream_t stream);

/* The Gaussian test matrix the range finder draws: Omega (n x l, element type
 * of problem->dtype), from the generator contract documented in the library's
 * design notes (Philox4x64-10, Box-Muller).  For parity tests. */
rsvd_status rsvd_draw_omega(rsvd_handle handle, const rsvd_problem* problem,
                            void* Omega, hipStream_t stream);

/* The SRFT ingredients the range finder draws (Section 4.6): the signs of D
 * (d: n doubles, +-1, device) and the sampled frequencies R (l distinct int32
 * in [0, n), device, in draw order), from the generator contract documented in
 * the library's design notes.  problem->sketch must be RSVD_SRFT.  For parity
 * tests. */
rsvd_status rsvd_draw_srft(rsvd_handle handle, const rsvd_problem* problem,
                           double* d, int32_t* R, hipStream_t stream);

/* CholeskyQR2 of a tall matrix on its own: Y (rows x l, element type of
 * problem->dtype, real) is overwritten by Q with Y = Q R; R (l x l, double,
 * upper triangular, positive diagonal) is written if non-NULL.  Uses problem->k
 * + problem->p as l and `rows` as the row count; needs
 * rsvd_workspace_bytes(problem) with problem->m >= rows. */
rsvd_status rsvd_orth(rsvd_handle handle, const rsvd_problem* problem,
                      int64_t rows, void* Y, double* R, void* ws,
                      size_t ws_bytes, hipStream_t stream);

/* --- Achievable peaks (measurement aids, not part of the method) --------- */

/* Read `bytes` (a multiple of 16) of the DEVICE buffer `buf` (16-byte aligned)
 * once, with 16-byte loads over 2048 workgroups of 256 threads and eight loads
 * in flight per thread, and write one float per workgroup to the DEVICE array
 * `sink` (2048 floats).  Enqueued on `stream`; the caller times it.  The
 * streaming-read rate it reaches is the HBM ceiling the benchmark reports
 * beside the datasheet's. */
rsvd_status rsvd_probe_hbm_read(const void* buf, size_t bytes, float* sink, hipStream_t stream);

/* `blocks` workgroups of four waves, each wave issuing `iters` rounds of four
 * independent MFMA accumulations on register operands -- kind 0: BF16
 * 32x32x16 (32768 flops each), 1: FP32 32x32x2 (4096), 2: FP64 16x16x4
 * (2048) -- then writing 256 floats per workgroup to the DEVICE array `sink`.
 * Enqueued on `stream`; the caller times it.  Its rate is the MFMA ceiling the
 * benchmark reports beside the datasheet's. */
rsvd_status rsvd_probe_mfma(int32_t kind, int64_t iters, int64_t blocks, float* sink, hipStream_t stream);

/* --- Kernel timing (a profiling aid) ------------------------------------ */

/* Kernel families that can be timed. */
enum {
  RSVD_KERNEL_STREAM_NN = 0,  /* GEMMs that stream A: A X (sketch, power steps) */
  RSVD_KERNEL_STREAM_TN = 1,  /* GEMMs that stream A: A^T X (power steps, projection) */
  RSVD_KERNEL_SMALL_GEMM = 2, /* Y R^-1 and the lifts (K = l) */
  RSVD_KERNEL_GRAM = 3,       /* block Gram + reduction */
  RSVD_KERNEL_CHOL = 4,       /* l x l Cholesky with inverse */
  RSVD_KERNEL_JACOBI = 5,     /* l x l one-sided Jacobi */
  RSVD_KERNEL_PACK = 6,       /* packing of the l-column operand before a streaming GEMM */
  RSVD_KERNEL_SRFT = 7,       /* SRFT sketch: one FFT per row of A D, sampled */
  RSVD_KERNEL_EIG = 8,        /* l x l symmetric eigensolver of B B* (small SVD of FP32 data) */
  RSVD_KERNEL_GSRFT = 9,      /* the Givens chains in front of the SRFT, one row of A at a time */
  RSVD_KERNEL_KINDS = 10
};

/* capacity > 0: create `capacity` pairs of hipEvents (an allocation made here,
 * never inside the hot-path calls) and bracket every later launch of the
 * families above with two events recorded on the launch's stream, until the
 * pairs run out.  capacity == 0: stop timing and release the events. */
rsvd_status rsvd_profile_enable(rsvd_handle handle, int32_t capacity);

/* Restrict timing to the families whose bit (1 << family) is set in `mask`
 * (all families after rsvd_profile_enable): a timed region that brackets only
 * the launches of interest pays for fewer events. */
rsvd_status rsvd_profile_select(rsvd_handle handle, uint32_t mask);

/* Wait for the recorded events; for each family f write the number of timed
 * launches to launches[f] and their summed durations (ms) to total_ms[f]
 * (arrays of RSVD_KERNEL_KINDS host elements); then forget the records. */
rsvd_status rsvd_profile_read(rsvd_handle handle, int32_t* launches,
                              double* total_ms);

/* Synchronizes `stream`, returns the accumulated device status bits in *flags
 * (RSVD_FLAG_*) and clears them. */
rsvd_status rsvd_device_status(rsvd_handle handle, hipStream_t stream,
                               int32_t* flags);

#ifdef __cplusplus
}
#endif

#endif /* RSVD_H */
