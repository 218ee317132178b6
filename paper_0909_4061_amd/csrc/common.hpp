// Shared declarations of the gfx950 randomized-SVD library: vector types for
// the MFMA builtins, the parameter blocks of every kernel family, and the
// host-side launchers that api.cpp drives.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rsvd.h"

namespace rsvd {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Arithmetic of the GEMMs that stream A.
enum Prec { PREC_NATIVE = 0, PREC_BF16 = 1, PREC_BF16X3 = 2 };

// ---------------------------------------------------------------------------
// Tall-skinny GEMM: C (rows x ncols) = op(A) * X, op(A) = A (NN) or A^T (TN).
// A is row-major with leading dimension lda.  NN: A is rows x K.  TN: A is
// K x rows.  X is K x ncols row-major (ldx).  With S == 1 the result goes to
// `out` (rows x ncols, ldo, element type of A).  With S > 1 the K range is split
// into S chunks of kchunk and chunk s writes its partial product to
// part[s][row][0..Lp) (element type of A, Lp = ncols rounded up to the tile
// width); the partials are summed by a reduction kernel in a fixed order.
struct GemmParams {
  const void* A;
  int64_t lda;
  int64_t rows;
  int64_t K;
  const void* X;
  int64_t ldx;
  int32_t ncols;
  int32_t Lp;
  void* out;
  int64_t ldo;
  void* part;
  int64_t kchunk;
  int32_t S;
  int32_t vec;          // 1: A rows (NN) / A columns (TN) allow 16-byte loads
  int32_t accum;        // 1: out += op(A) X (S == 1 only); 0: out = op(A) X
  const int32_t* gate;  // if non-null and *gate == 0 the kernel does nothing
  int32_t narrow;       // FP32 native, S == 1, K <= 256: 32-row blocks (more workgroups for one product)
  void* pack;           // the A-streaming kernels: X packed by pack_x (stream_pack_bytes(K, Lp) bytes)
  int32_t wide;         // the A-streaming BF16 kernels: Lp > 128 allowed, 128-column chunks per workgroup
};

// Tile geometry of each GEMM variant (rows of C per workgroup, K per stage).
struct GemmTile { int bm, bk, lp_mult; };
GemmTile gemm_tile(int dtype, int prec);

hipError_t launch_gemm(int dtype, int prec, bool trans, const GemmParams& p, hipStream_t st);

// FP32-data GEMMs that stream A (FP32 MFMA or BF16 / bf16x3 MFMA): X is first
// packed into `pack` (stream_pack_bytes(K, Lp) bytes) by a small kernel.
int64_t stream_pack_bytes(int64_t K, int32_t Lp);
bool stream_params_ok(int prec, const GemmParams& p);
hipError_t launch_pack_x(int prec, const GemmParams& p, hipStream_t st);
hipError_t launch_stream_gemm(int prec, bool trans, const GemmParams& p, hipStream_t st);

// ---------------------------------------------------------------------------
// Gram matrices and CholeskyQR.
struct GramParams {
  const void* part;      // S x rows x Lp split-K partial products (summed by sum_parts)
  int32_t S;
  int32_t Lp;
  const void* yin;       // rows x l read by the Gram, leading dimension ldy
  void* yout;            // rows x l written by sum_parts, leading dimension ldy
  int64_t ldy;
  int64_t rows;
  int32_t l;
  int32_t Lg;            // l rounded up to 16
  double* gpart;         // nblk x Lg x Lg: upper 16x16 tiles of each chunk's Gram
  const int32_t* gate;
  int32_t tgroups;       // workgroup b: row chunk b / tgroups, tiles t = b % tgroups (mod tgroups)
  int32_t chunk;         // rows per chunk, a multiple of GRAM_ROWS
};
constexpr int GRAM_ROWS = 64;  // rows of Y staged at a time by a Gram workgroup
// Chunks and tile groups of the Gram of `rows` rows (returns the chunk count,
// which is the number of partial Grams).  wide: split the tiles of each chunk
// over workgroups so that a single Gram fills the chip with few partials;
// otherwise one workgroup per two GRAM_ROWS-row stages with every tile (a
// batch of Grams fills the chip by itself; 64 and 512 rows measured slower,
// 256 the same).
int64_t gram_geometry(int64_t rows, int32_t Lg, bool wide, int32_t* tgroups, int32_t* chunk);
// yout (rows x l, leading dimension ldy) = sum over s of the S split-K partials
// part[s] (rows x Lp), in the order s = 0, 1, ...
hipError_t launch_sum_parts(int dtype, const GramParams& p, hipStream_t st);
bool sum_parts_ok(int dtype, const GramParams& p);
int64_t sum_parts_blocks(int dtype, const GramParams& p);

hipError_t launch_gram_partial(int dtype, const GramParams& p, hipStream_t st);
hipError_t launch_gram_reduce(const double* gpart, int64_t nblk, int32_t Lg, double* G,
                              int32_t* status, const int32_t* gate, hipStream_t st);

struct CholParams {
  const double* G;      // Lg x Lg, upper triangle read
  int32_t Lg;
  int32_t l;
  int64_t rows;         // row count of the matrix whose Gram G is (for the shift)
  double* R;            // l x l upper triangular, positive diagonal (may be null)
  double* Rinv;         // l x l, R^-1 (may be null)
  void* RinvT;          // l x l, R^-1 rounded to the element type (may be null)
  int32_t dtype;
  int32_t* shifted;     // set to 1 when a shift was needed (may be null)
  int32_t reset_shifted;  // 1: *shifted is first cleared (the first factorization of a CholeskyQR)
  int32_t* status;      // handle status word (RSVD_FLAG_*)
  const int32_t* gate;
};
hipError_t launch_chol(const CholParams& p, hipStream_t st);

// R = R2 * R1 for upper triangular l x l factors (FP64).
hipError_t launch_trmm_upper(const double* R2, const double* R1, double* R, int32_t l,
                             const int32_t* gate, hipStream_t st);

// ---------------------------------------------------------------------------
// Small SVD: one-sided Jacobi on C = R^T (l x l) with R from the Cholesky of B B*.
struct JacobiParams {
  const double* R;      // l x l upper triangular
  int32_t l;
  int32_t k;
  int32_t dtype;
  double* Uh;           // l x l left singular vectors of R^T, by descending sigma
  double* sig;          // l singular values, descending
  void* XU;             // l x k: Uh[:, :k] in the element type
  void* XV;             // l x k: Uh[:, :k] diag(1/sigma) in the element type
  void* S;              // k singular values in the element type
  int32_t* status;
  int32_t* sweeps;      // if non-null: number of sweeps run (diagnostic)
};
hipError_t launch_jacobi(const JacobiParams& p, hipStream_t st);

// ---------------------------------------------------------------------------
// Achievable-peak probes (measurement aids).
hipError_t launch_hbm_read(const void* buf, size_t bytes, float* sink, hipStream_t st);
hipError_t launch_mfma_loop(int kind, int64_t iters, int64_t blocks, float* sink, hipStream_t st);

// ---------------------------------------------------------------------------
// Random test matrices (counter-based Philox4x64-10).
hipError_t launch_omega(int dtype, void* omega, int64_t n, int32_t l, uint64_t seed,
                        uint64_t stream_id, hipStream_t st);
hipError_t launch_srft_draw(double* d, int32_t* R, int64_t n, int32_t l, uint64_t seed,
                            uint64_t stream_id, hipStream_t st);

// Givens-chain structured test matrix: the tables of its two chains (c = 0:
// D', Theta; c = 1: D'', Theta') in a workspace region of gsrft_table_bytes(n,
// element size), and the pretransform out (m x n, row stride n) = A D'' Theta'
// D' Theta, which the SRFT kernels then sketch.  n a power of two, 8 <= n <=
// 16384 (FP32) or 8192 (FP64): a row and its gathered copy in one workgroup's LDS.
constexpr int GSRFT_MAX_N = 16384;
template <typename T>
struct GsrftTables {
  uint64_t* key[2];  // sort keys of the permutations
  T* sign[2];        // +-1
  T* cs[2];          // (cos theta_j, sin theta_j) pairs, j < n - 1; (1, 0) at j = n - 1
  T* psign[2];       // sign[pi(j)]
  int32_t* perm[2];  // pi: (x Pi)_j = x_pi(j)
};
size_t gsrft_table_bytes(int64_t n, int esize);
bool gsrft_shape_ok(int dtype, int64_t n);
hipError_t launch_gsrft_draw(int dtype, void* tables, int64_t n, uint64_t seed, uint64_t sid, hipStream_t st);
hipError_t launch_gsrft_rows(int dtype, const void* A, int64_t lda, int64_t m, int64_t n, void* tables, void* out,
                             hipStream_t st);

// SRFT sketch Y (m x l, row-major) = A Omega for the real SRFT with signs d
// and sampled frequencies R; n = 2^(LOGN+1) with 2 <= LOGN <= SRFT_MAX_LOGN_*.
constexpr int SRFT_MAX_LOGN_F32 = 13;  // n <= 16384
constexpr int SRFT_MAX_LOGN_F64 = 12;  // n <= 8192
hipError_t launch_srft_rows(int dtype, const void* A, int64_t lda, int64_t m, int64_t n, int32_t l,
                            const double* d, const int32_t* R, void* Y, hipStream_t st);

// ---------------------------------------------------------------------------
// Batched launches: one grid runs one kernel family on many independent
// problems.  Block b of the grid runs local block bm[b].local of problem
// bm[b].item, whose parameter block is ps[bm[b].item]; both arrays live in
// device memory.  The per-problem block count of a family is what its
// single-problem launcher would launch.
struct BlockMap { int32_t item, local; };

// ---------------------------------------------------------------------------
// Symmetric eigensolver of the FP64 Gram W = B B* (small SVD of FP32 data):
// stage 0 tridiagonalizes W (one workgroup), stage 1 finds each eigenpair of
// T and transforms it back (one wave per eigenvalue), stage 2 orthogonalizes
// clustered and flagged columns (one workgroup).  Outputs as JacobiParams.
struct EigParams {
  const double* G;  // Lg x Lg, the upper triangle of W (row i, columns >= i)
  int32_t Lg;
  int32_t l;
  int32_t k;
  int32_t dtype;    // element type of XU, XV, S
  double* V;        // l x EIG_LDV workspace: row i = Householder vector of step i
  double* tri;      // 3 l workspace: diagonal d, off-diagonal e, tau
  double* lam;      // l workspace: eigenvalues of W, descending
  double* Z;        // l x l workspace: row j = eigenvector j
  int32_t* flag;    // l workspace
  double* tnorm;    // 1 workspace: Gershgorin bound of ||T||
  double* Uh;       // l x l: column j = eigenvector j (descending)
  double* sig;      // l: sqrt(max(lambda_j, 0))
  void* XU;         // l x k: Uh[:, :k] in the element type
  void* XV;         // l x k: Uh[:, :k] diag(1/sig) in the element type
  void* S;          // k
  int32_t* status;
};
constexpr int EIG_LDV = 128;  // row stride of the reflectors (any compiled variant writes whole rows)
int eig_variant(int32_t l);
int64_t eig_blocks(int stage, const EigParams& p);
hipError_t launch_eig(int stage, const EigParams& p, hipStream_t st);
// Two independent problems of the same l, one launch per stage.
hipError_t launch_eig_pair(int stage, const EigParams& a, const EigParams& b, hipStream_t st);
hipError_t launch_eig_batched(int stage, int variant, const EigParams* ps, const BlockMap* bm, int64_t nblocks,
                              hipStream_t st);

// Stage B for symmetric / psd A (k_sym.hip).  sym_gram: G (FP64, upper
// triangle, stride Lg) = (B + B^T) / 2 of an l x l matrix B (element type,
// row stride ldb).  eig_pick: the k kept eigenpairs of an eigensolver run
// (lam descending by value, Uh[i * l + j] = component i of eigenvector j):
// by magnitude (Lam = lambda, XU = the matching columns, l x k) or by value
// (Lam = sig^2 for the first k).
struct SymGramParams {
  const void* B;
  int32_t dtype;
  int32_t l;
  int32_t ldb;
  int32_t Lg;
  double* G;
};
struct EigPickParams {
  const double* lam;
  const double* Uh;
  const double* sig;
  int32_t l;
  int32_t k;
  int32_t by_magnitude;
  int32_t dtype;
  void* Lam;  // k, element type
  void* XU;   // l x k, element type (magnitude order only; may be null)
};
hipError_t launch_sym_gram(const SymGramParams& p, hipStream_t st);
// C = X1^T X2 (c1 x c2) over `rows` rows: partials of CROSS_ROWS rows into
// part (nblk blocks of Lg x Lg FP64), then their sum into out (element type,
// sym == 0) or its symmetric part into G (FP64 upper triangle, sym == 1).
constexpr int CROSS_ROWS = 64;
struct CrossParams {
  const void* X1;
  int64_t ld1;
  const void* X2;
  int64_t ld2;
  int64_t rows;
  int32_t c1, c2;
  int32_t dtype;
  int32_t Lg;
  double* part;
  int64_t nblk;
  int32_t sym;
  void* out;
  int64_t ldo;
  double* G;
  int32_t out_f64;  // sym == 0: out holds doubles instead of the element type
};
int64_t cross_blocks(int64_t rows);
// X_ij /= (d2_i + d1_j) for an l x l FP64 matrix X (row stride ld): the
// diagonalized Sylvester equation of the two-sided single pass.
hipError_t launch_sylv_div(double* X, int64_t ld, const double* d2, const double* d1, int32_t l, hipStream_t st);
hipError_t launch_cross(const CrossParams& p, hipStream_t st);
hipError_t launch_eig_pick(const EigPickParams& p, hipStream_t st);

struct GramReduceParams {
  const double* gpart;
  int64_t nblk;
  int32_t Lg;
  double* G;
  int32_t* status;
  const int32_t* gate;
};
struct OmegaParams {
  void* omega;
  int64_t n;
  int32_t l;
  uint64_t seed, sid;
};
struct TrmmParams {  // R = R2 * R1, upper triangular l x l (FP64)
  const double* R2;
  const double* R1;
  double* R;
  int32_t l;
  const int32_t* gate;
};
struct CopyParams {
  const double* src;
  double* dst;
  int64_t count;
  const int32_t* gate;
};

int64_t gemm_blocks(int dtype, int prec, const GemmParams& p);
int64_t gram_partial_blocks(const GramParams& p);
int64_t gram_reduce_blocks(const GramReduceParams& p);
int64_t omega_blocks(const OmegaParams& p);
int64_t trmm_blocks(const TrmmParams& p);
int64_t copy_blocks(const CopyParams& p);

hipError_t launch_gemm_batched(int dtype, int prec, bool trans, const GemmParams* ps, const BlockMap* bm,
                               int64_t nblocks, hipStream_t st);
hipError_t launch_gram_partial_batched(int dtype, const GramParams* ps, const BlockMap* bm, int64_t nblocks,
                                       hipStream_t st);
hipError_t launch_gram_reduce_batched(const GramReduceParams* ps, const BlockMap* bm, int64_t nblocks,
                                      hipStream_t st);
hipError_t launch_chol_batched(const CholParams* ps, const BlockMap* bm, int64_t nblocks, hipStream_t st);
// Jacobi variants: the largest l a kernel instance holds (32, 64, 80, 96 or 128).
int jacobi_variant(int32_t l);
hipError_t launch_jacobi_batched(int variant, const JacobiParams* ps, const BlockMap* bm, int64_t nblocks,
                                 hipStream_t st);
hipError_t launch_omega_batched(int dtype, const OmegaParams* ps, const BlockMap* bm, int64_t nblocks,
                                hipStream_t st);
hipError_t launch_trmm_batched(const TrmmParams* ps, const BlockMap* bm, int64_t nblocks, hipStream_t st);
hipError_t launch_copy_batched(const CopyParams* ps, const BlockMap* bm, int64_t nblocks, hipStream_t st);
hipError_t launch_sum_parts_batched(int dtype, const GramParams* ps, const BlockMap* bm, int64_t nblocks,
                                    hipStream_t st);
int64_t pack_x_blocks(const GemmParams& p);
int64_t stream_gemm_blocks(const GemmParams& p);
hipError_t launch_pack_x_batched(int prec, const GemmParams* ps, const BlockMap* bm, int64_t nblocks,
                                 hipStream_t st);
hipError_t launch_stream_gemm_batched(int prec, bool trans, bool wide, const GemmParams* ps, const BlockMap* bm,
                                      int64_t nblocks, hipStream_t st);

// ---------------------------------------------------------------------------
// Adjoint pieces (l x l algebra in FP64, strided copies).
struct SvdAdjParams {
  const double* Uh;   // l x l, U~ of the small SVD (row-major)
  const double* sig;  // l singular values
  const void* T1;     // l x k, B gV        (element type)
  const void* T2;     // l x k, Q^T gU      (element type)
  const void* gS;     // k                  (element type)
  int32_t l, k, dtype;
  double* Z;          // l x l: S^-1 (C - P1 S^-1)
  double* M2;         // k x l: S_k^-1 U~_k^T
  double* Ukt;        // k x l: U~_k^T
};
struct Copy2dParams {
  const void* src;
  int32_t src_dtype;
  int64_t lds;
  void* dst;
  int32_t dst_dtype;
  int64_t ldd;
  int64_t rows, cols;  // of the source block
  int32_t trans;       // 1: dst = src^T
  int32_t negate;      // 1: dst = -src (or -src^T)
};
struct QrSymParams {  // S = sym(-M^T) (FP64, l x l) for M = Q^T gQ (element type)
  const void* M;
  int32_t dtype, l;
  double* S;
};
struct TriInvParams {  // Rinv = R^-1, R upper triangular l x l (FP64), l <= 128
  const double* R;
  double* Rinv;
  int32_t l;
};
int64_t svd_adj_coef_blocks(const SvdAdjParams& p);
int64_t qr_adj_sym_blocks(const QrSymParams& p);
int64_t copy2d_blocks(const Copy2dParams& p);
bool svd_adj_coef_ok(const SvdAdjParams& p);
bool tri_inv_ok(const TriInvParams& p);
hipError_t launch_svd_adj_coef(const SvdAdjParams& p, hipStream_t st);
hipError_t launch_qr_adj_sym(const QrSymParams& p, hipStream_t st);
hipError_t launch_tri_inv_upper(const TriInvParams& p, hipStream_t st);
hipError_t launch_copy2d(const Copy2dParams& p, hipStream_t st);
hipError_t launch_svd_adj_coef_batched(const SvdAdjParams* ps, const BlockMap* bm, int64_t nblocks, hipStream_t st);
hipError_t launch_qr_adj_sym_batched(const QrSymParams* ps, const BlockMap* bm, int64_t nblocks, hipStream_t st);
hipError_t launch_tri_inv_upper_batched(const TriInvParams* ps, const BlockMap* bm, int64_t nblocks,
                                        hipStream_t st);
hipError_t launch_copy2d_batched(const Copy2dParams* ps, const BlockMap* bm, int64_t nblocks, hipStream_t st);

// Small utilities.
hipError_t launch_copy_f64(const double* src, double* dst, int64_t count, const int32_t* gate, hipStream_t st);

}  // namespace rsvd
