// The SVD of the small matrix B (Algorithm 5.1, step 2), in FP64.
//
// The host first forms the l x l Gram B B* and its Cholesky factor R (so that
// R^T R = B B*).  The left singular vectors and singular values of B are those
// of C = R^T:  C C^T = R^T R = B B*.  One-sided (Hestenes) Jacobi rotates pairs
// of columns of C until all columns are mutually orthogonal; then C J = U~ S,
// so U~ = normalized columns and S = column norms.  The right factor J is not
// needed: the right singular vectors follow as V = B* U~ S^-1, computed by the
// lift GEMM (B* is the stored Bt).
//
// One workgroup of 512 threads holds C column-major in LDS.  Each round of a
// sweep rotates l/2 disjoint column pairs chosen by the round-robin (circle)
// ordering, one pair per 8-lane group; a sweep is l - 1 rounds (l rounded up
// to even, with a zero column when l is odd), so every pair meets once.  A
// pair is rotated when |c_i . c_j| > tol sqrt(|c_i|^2 |c_j|^2); the workgroup
// stops after a sweep with no rotation.
#include <float.h>

#include "common.hpp"

namespace rsvd {

namespace {

constexpr int JAC_MAXL = 128;
constexpr int JAC_LDC = JAC_MAXL + 2;  // even: 16-byte aligned column starts
constexpr int JAC_MAX_SWEEPS = 40;

// Move a double across lanes of a 16-lane DPP row.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over an aligned group of 8 lanes.  Mirror within the half-row, then
// swaps within quads: every lane adds the same operands in the same pairs, so
// all 8 lanes hold bitwise-identical sums (and take identical rotation
// decisions).
__device__ inline double group8_sum(double v) {
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  return v;
}

__device__ __forceinline__ void jacobi_body(const JacobiParams& p, const int bid) {
  (void)bid;  // one workgroup per matrix
  __shared__ __attribute__((aligned(16))) double Cs[JAC_MAXL * JAC_LDC];  // column c at Cs[c * JAC_LDC + row]
  __shared__ double sig_s[JAC_MAXL];
  __shared__ int rank_s[JAC_MAXL];
  __shared__ int rotated;
  const int tid = threadIdx.x;
  const int l = p.l;
  const int le = l + (l & 1);
  const int P = le / 2;

  // column c of C = R^T is row c of R
  for (int idx = tid; idx < le * JAC_LDC; idx += 512) {
    const int c = idx / JAC_LDC, i = idx - c * JAC_LDC;
    Cs[idx] = (c < l && i < l) ? p.R[(int64_t)c * l + i] : 0.0;
  }
  if (tid == 0) rotated = 1;
  __syncthreads();

  const int grp = tid >> 3, gl = tid & 7;
  const double tol = (double)l * DBL_EPSILON;
  int sweep = 0;
  for (; sweep < JAC_MAX_SWEEPS; ++sweep) {
    if (rotated == 0) break;  // read after the barrier that ended the last sweep
    __syncthreads();
    if (tid == 0) rotated = 0;
    __syncthreads();
    int any = 0;
    for (int rnd = 0; rnd < le - 1; ++rnd) {
      if (grp < P) {
        // positions grp and le-1-grp; column at position x is 0 for x == 0,
        // else 1 + (x - 1 + rnd) mod (le - 1)
        const int xa = grp, xb = le - 1 - grp;
        const int ca = xa == 0 ? 0 : 1 + (xa - 1 + rnd) % (le - 1);
        const int cb = 1 + (xb - 1 + rnd) % (le - 1);
        double* col_a = Cs + ca * JAC_LDC;
        double* col_b = Cs + cb * JAC_LDC;
        // rows 16 r + 2 gl and 16 r + 2 gl + 1 of each column (rows past l are zeros)
        typedef double d2 __attribute__((ext_vector_type(2)));
        double x[JAC_MAXL / 8], y[JAC_MAXL / 8];
#pragma unroll
        for (int r = 0; r < JAC_MAXL / 16; ++r) {
          const d2 xa = *reinterpret_cast<const d2*>(col_a + 16 * r + 2 * gl);
          const d2 yb = *reinterpret_cast<const d2*>(col_b + 16 * r + 2 * gl);
          x[2 * r] = xa[0];
          x[2 * r + 1] = xa[1];
          y[2 * r] = yb[0];
          y[2 * r + 1] = yb[1];
        }
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int r = 0; r < JAC_MAXL / 8; ++r) {
          al += x[r] * x[r];
          be += y[r] * y[r];
          ga += x[r] * y[r];
        }
        al = group8_sum(al);
        be = group8_sum(be);
        ga = group8_sum(ga);
        if (ca < l && cb < l && fabs(ga) > tol * sqrt(al * be) && al > 0.0 && be > 0.0) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t);
          const double sn = cs * t;
#pragma unroll
          for (int r = 0; r < JAC_MAXL / 16; ++r) {
            *reinterpret_cast<d2*>(col_a + 16 * r + 2 * gl) =
                d2{cs * x[2 * r] - sn * y[2 * r], cs * x[2 * r + 1] - sn * y[2 * r + 1]};
            *reinterpret_cast<d2*>(col_b + 16 * r + 2 * gl) =
                d2{sn * x[2 * r] + cs * y[2 * r], sn * x[2 * r + 1] + cs * y[2 * r + 1]};
          }
          any = 1;
        }
      }
      __syncthreads();
    }
    if (any) rotated = 1;  // benign race: every writer stores 1
    __syncthreads();
  }
  if (tid == 0 && sweep >= JAC_MAX_SWEEPS && rotated) atomicOr(p.status, (int32_t)RSVD_FLAG_NOCONV);
  if (tid == 0 && p.sweeps) *p.sweeps = sweep;

  // singular values = column norms; rank by descending value (ties: lower index first)
  if (tid < l) {
    double s2 = 0.0;
    for (int i = 0; i < l; ++i) s2 += Cs[tid * JAC_LDC + i] * Cs[tid * JAC_LDC + i];
    sig_s[tid] = sqrt(s2);
  }
  __syncthreads();
  if (tid < l) {
    const double me = sig_s[tid];
    int rk = 0;
    for (int c = 0; c < l; ++c) {
      const double o = sig_s[c];
      rk += (o > me) || (o == me && c < tid);
    }
    rank_s[tid] = rk;
  }
  __syncthreads();
  for (int idx = tid; idx < l * l; idx += 512) {
    const int c = idx / l, i = idx - c * l;  // element i of column c
    const int rk = rank_s[c];
    const double sg = sig_s[c];
    const double u = sg > 0.0 ? Cs[c * JAC_LDC + i] / sg : 0.0;
    p.Uh[(int64_t)i * l + rk] = u;
    if (rk < p.k) {
      const double v = sg > 0.0 ? u / sg : 0.0;
      if (p.dtype == RSVD_F64) {
        ((double*)p.XU)[(int64_t)i * p.k + rk] = u;
        ((double*)p.XV)[(int64_t)i * p.k + rk] = v;
      } else {
        ((float*)p.XU)[(int64_t)i * p.k + rk] = (float)u;
        ((float*)p.XV)[(int64_t)i * p.k + rk] = (float)v;
      }
    }
  }
  if (tid < l) {
    const int rk = rank_s[tid];
    p.sig[rk] = sig_s[tid];
    if (rk < p.k) {
      if (p.dtype == RSVD_F64) ((double*)p.S)[rk] = sig_s[tid];
      else ((float*)p.S)[rk] = (float)sig_s[tid];
    }
  }
}

__global__ __launch_bounds__(512) void jacobi_kernel(const JacobiParams p) { jacobi_body(p, blockIdx.x); }

__global__ __launch_bounds__(512) void jacobi_batched(const JacobiParams* __restrict__ ps, const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  jacobi_body(ps[b.item], b.local);
}

}  // namespace

hipError_t launch_jacobi(const JacobiParams& p, hipStream_t st) {
  if (p.l < 1 || p.l > JAC_MAXL || p.k < 1 || p.k > p.l) return hipErrorInvalidValue;
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(512), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_jacobi_batched(const JacobiParams* ps, const BlockMap* bm, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_batched, dim3((unsigned)nblocks), dim3(512), 0, st, ps, bm);
  return hipGetLastError();
}

}  // namespace rsvd
