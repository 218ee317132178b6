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
// One workgroup holds C column-major in LDS.  Each round of a sweep rotates
// l/2 disjoint column pairs chosen by the round-robin (circle) ordering, one
// pair per 4-lane group; a sweep is l - 1 rounds (l rounded up to even, with a
// zero column when l is odd), so every pair meets once.  A pair is rotated
// when |c_i . c_j| > tol sqrt(|c_i|^2 |c_j|^2); the workgroup stops after a
// sweep with no rotation.  The squared column norms are formed exactly in the
// first round of every sweep and carried through its other rounds (a rotation
// changes them by -t c_i . c_j and +t c_i . c_j), so a round forms one dot
// product per pair instead of three.  A single matrix runs eight lanes per
// pair (two waves per SIMD, which hide each other's LDS and FP64 latencies);
// a batch runs four (several workgroups share a CU).  The kernel is compiled
// for l <= 32, 64, 80, 96 and 128: a smaller variant holds fewer rows per lane
// (rows past l are zeros but still cost work) and less LDS (more workgroups
// per CU in a batch).
#include <float.h>

#include "common.hpp"

namespace rsvd {

namespace {

constexpr int JAC_MAX_SWEEPS = 40;

// Move a double across lanes of a 16-lane DPP row.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over an aligned group of 4, 8 or 16 lanes: two swaps within the quad,
// then the other quad's sum by a mirror within the half-row (8 lanes), then
// the other half-row's by a mirror within the row (16 lanes).  Every lane
// adds the same operands in the same pairs (the last addition in either
// order, which is exact to the same bits), so all lanes of a group hold
// bitwise-identical sums and take identical rotation decisions.
template <int LPP>
__device__ inline double group_sum(double v) {
  v += dpp_f64<0x4E>(v);  // quad_perm [2,3,0,1]
  v += dpp_f64<0xB1>(v);  // quad_perm [1,0,3,2]
  if (LPP >= 8) v += dpp_f64<0x141>(v);   // row_half_mirror: lane i <- lane 7 - i of its 8
  if (LPP == 16) v += dpp_f64<0x140>(v);  // row_mirror: lane i <- lane 15 - i of its 16
  return v;
}

// 1/x and 1/sqrt(x) from the hardware estimates and two Newton steps each
// (quadratic convergence from the estimates' ~2^-22 relative error to the
// FP64 rounding level).  The rotation below needs c^2 + s^2 = 1 to rounding,
// not correctly rounded quotients, and these short chains are a fraction of
// the latency of IEEE division and square root.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x * y, y, 1.0);  // 1 - x y^2
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// One workgroup of MAXL / 2 * LPP threads per matrix (l <= MAXL): MAXL / 2
// column pairs per round, LPP lanes per pair, each lane holding MAXL / LPP
// rows of both columns in registers.
template <int MAXL, int LPP>
constexpr int jac_threads() { return MAXL / 2 * LPP; }

template <int MAXL, int LPP>
__device__ __forceinline__ void jacobi_body(const JacobiParams& p, const int bid) {
  (void)bid;  // one workgroup per matrix
  // Column stride: 16-byte aligned and, modulo the 256-byte bank width, 64
  // bytes (four lanes per pair; 192 serves as well) or 128 bytes (eight), so
  // the 16-byte accesses of the groups of one wave, consecutive columns, fall
  // on distinct bank slots (sixteen lanes read 256 contiguous bytes, one per
  // bank, at any stride).  With eight lanes, MAXL = 80 is already 128 bytes
  // modulo 256; MAXL + 16 would put every group on the same half.
  constexpr int LDC = LPP == 8 ? (MAXL % 32 == 16 ? MAXL : MAXL + 16) : MAXL + 8;
  static_assert((LDC * 8) % 256 == (LPP == 8 ? 128 : 64) || (LPP == 4 && (LDC * 8) % 256 == 192),
                "column stride off the bank pattern");
  constexpr int THREADS = jac_threads<MAXL, LPP>();
  constexpr int RPL = MAXL / LPP;  // rows per lane
  typedef double d2 __attribute__((ext_vector_type(2)));
  __shared__ __attribute__((aligned(16))) double Cs[MAXL * LDC];  // column c at Cs[c * LDC + row]
  __shared__ double sig_s[MAXL];
  __shared__ double nrm[MAXL];  // squared column norms, exact at the start of a sweep
  __shared__ int rank_s[MAXL];
  __shared__ double sgn_s[MAXL];
  __shared__ int rotated;
  const int tid = threadIdx.x;
  const int l = p.l;
  const int le = l + (l & 1);
  const int P = le / 2;

  // column c of C = R^T is row c of R
  for (int idx = tid; idx < le * LDC; idx += THREADS) {
    const int c = idx / LDC, i = idx - c * LDC;
    Cs[idx] = (c < l && i < l) ? p.R[(int64_t)c * l + i] : 0.0;
  }
  if (tid == 0) rotated = 1;
  __syncthreads();

  const int grp = tid / LPP, gl = tid % LPP;
  // Stopping threshold on |c_i . c_j| / (|c_i| |c_j|): the unit roundoff of
  // the output type (FP32 outputs cannot show a smaller loss of
  // orthogonality), l eps for FP64 outputs.
  const double tol = p.dtype == RSVD_F64 ? (double)l * DBL_EPSILON : (double)FLT_EPSILON;
  // Round-robin (circle) ordering: position 0 holds column 0; position x > 0
  // holds column 1 + (x - 1 + rnd) mod (le - 1).  This group owns positions
  // grp and le - 1 - grp; the offsets advance by one per round and return to
  // their start after a sweep of le - 1 rounds.
  const int ia0 = grp > 0 ? grp - 1 : 0;
  const int ib0 = le - 2 - grp;
  int sweep = 0;
  for (; sweep < JAC_MAX_SWEEPS; ++sweep) {
    if (rotated == 0) break;  // read after the barrier that ended the last sweep
    __syncthreads();
    if (tid == 0) rotated = 0;
    __syncthreads();
    int any = 0;
    int ia = ia0, ib = ib0;
    for (int rnd = 0; rnd < le - 1; ++rnd) {
      if (grp < P) {
        const int ca = grp == 0 ? 0 : 1 + ia;
        const int cb = 1 + ib;
        double* col_a = Cs + ca * LDC;
        double* col_b = Cs + cb * LDC;
        // rows 2 LPP r + 2 gl and 2 LPP r + 2 gl + 1 of each column (rows past l are zeros)
        double x[RPL], y[RPL];
#pragma unroll
        for (int r = 0; r < RPL / 2; ++r) {
          const d2 xa = *reinterpret_cast<const d2*>(col_a + 2 * LPP * r + 2 * gl);
          const d2 yb = *reinterpret_cast<const d2*>(col_b + 2 * LPP * r + 2 * gl);
          x[2 * r] = xa[0];
          x[2 * r + 1] = xa[1];
          y[2 * r] = yb[0];
          y[2 * r + 1] = yb[1];
        }
        // The first round of a sweep forms every squared column norm exactly;
        // later rounds carry them (a rotation maps al, be to al - t ga, be + t ga)
        // and form only the cross product.  Four partial sums per product keep
        // the dependent chains short.
        double al, be, ga;
        if (rnd == 0) {
          double al4[4] = {0.0, 0.0, 0.0, 0.0}, be4[4] = {0.0, 0.0, 0.0, 0.0}, ga4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int r = 0; r < RPL; ++r) {
            al4[r & 3] += x[r] * x[r];
            be4[r & 3] += y[r] * y[r];
            ga4[r & 3] += x[r] * y[r];
          }
          al = group_sum<LPP>((al4[0] + al4[1]) + (al4[2] + al4[3]));
          be = group_sum<LPP>((be4[0] + be4[1]) + (be4[2] + be4[3]));
          ga = group_sum<LPP>((ga4[0] + ga4[1]) + (ga4[2] + ga4[3]));
        } else {
          double ga4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int r = 0; r < RPL; ++r) ga4[r & 3] += x[r] * y[r];
          ga = group_sum<LPP>((ga4[0] + ga4[1]) + (ga4[2] + ga4[3]));
          al = nrm[ca];
          be = nrm[cb];
        }
        // rotate when |ga| > tol sqrt(al be), tested as ga^2 > tol^2 al be
        const bool rot = ca < l && cb < l && ga * ga > tol * tol * al * be && al > 0.0 && be > 0.0;
        if (rot) {
          const double zeta = (be - al) * rcp_nr(2.0 * ga);
          const double q = fma(zeta, zeta, 1.0);
          const double root = q * rsq_nr(q);  // sqrt(1 + zeta^2)
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) * rcp_nr(fabs(zeta) + root);
          const double cs = rsq_nr(fma(t, t, 1.0));
          const double sn = cs * t;
#pragma unroll
          for (int r = 0; r < RPL / 2; ++r) {
            *reinterpret_cast<d2*>(col_a + 2 * LPP * r + 2 * gl) =
                d2{cs * x[2 * r] - sn * y[2 * r], cs * x[2 * r + 1] - sn * y[2 * r + 1]};
            *reinterpret_cast<d2*>(col_b + 2 * LPP * r + 2 * gl) =
                d2{sn * x[2 * r] + cs * y[2 * r], sn * x[2 * r + 1] + cs * y[2 * r + 1]};
          }
          al = fma(-t, ga, al);
          be = fma(t, ga, be);
        }
        if (gl == 0 && (rot || rnd == 0)) {
          nrm[ca] = al;
          nrm[cb] = be;
        }
        any |= rot ? 1 : 0;
      }
      ia = ia + 1 == le - 1 ? 0 : ia + 1;
      ib = ib + 1 == le - 1 ? 0 : ib + 1;
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
    for (int i = 0; i < l; ++i) s2 += Cs[tid * LDC + i] * Cs[tid * LDC + i];
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
    // sign convention: the component of largest magnitude (the first of equals) is positive
    double mx = -1.0, piv = 1.0;
    for (int i = 0; i < l; ++i) {
      const double v = Cs[tid * LDC + i];
      if (fabs(v) > mx) {
        mx = fabs(v);
        piv = v;
      }
    }
    sgn_s[tid] = piv < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  for (int idx = tid; idx < l * l; idx += THREADS) {
    const int c = idx / l, i = idx - c * l;  // element i of column c
    const int rk = rank_s[c];
    const double sg = sig_s[c];
    const double u = sg > 0.0 ? sgn_s[c] * Cs[c * LDC + i] / sg : 0.0;
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

// Lanes per column pair: eight for a single matrix or a batch with fewer
// matrices than CUs (two waves per SIMD hide each other's LDS and FP64
// latencies), four in a larger batch (several workgroups per CU already do).
constexpr int JAC_LPP_SINGLE = 8;
constexpr int JAC_LPP_BATCH = 4;
constexpr int JAC_BATCH_WIDE = 256;  // batches below this many matrices take the single-matrix form

template <int MAXL>
__global__ __launch_bounds__((jac_threads<MAXL, JAC_LPP_SINGLE>())) void jacobi_kernel(const JacobiParams p) {
  jacobi_body<MAXL, JAC_LPP_SINGLE>(p, blockIdx.x);
}

template <int MAXL, int LPP>
__global__ __launch_bounds__((jac_threads<MAXL, LPP>())) void jacobi_batched(const JacobiParams* __restrict__ ps,
                                                                           const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  jacobi_body<MAXL, LPP>(ps[b.item], b.local);
}

}  // namespace

int jacobi_variant(int32_t l) { return l <= 32 ? 32 : (l <= 64 ? 64 : (l <= 80 ? 80 : (l <= 96 ? 96 : 128))); }

hipError_t launch_jacobi(const JacobiParams& p, hipStream_t st) {
  if (p.l < 1 || p.l > 128 || p.k < 1 || p.k > p.l) return hipErrorInvalidValue;
  switch (jacobi_variant(p.l)) {
    case 32: hipLaunchKernelGGL(jacobi_kernel<32>, dim3(1), dim3(jac_threads<32, JAC_LPP_SINGLE>()), 0, st, p); break;
    case 64: hipLaunchKernelGGL(jacobi_kernel<64>, dim3(1), dim3(jac_threads<64, JAC_LPP_SINGLE>()), 0, st, p); break;
    case 80: hipLaunchKernelGGL(jacobi_kernel<80>, dim3(1), dim3(jac_threads<80, JAC_LPP_SINGLE>()), 0, st, p); break;
    case 96: hipLaunchKernelGGL(jacobi_kernel<96>, dim3(1), dim3(jac_threads<96, JAC_LPP_SINGLE>()), 0, st, p); break;
    default:
      hipLaunchKernelGGL(jacobi_kernel<128>, dim3(1), dim3(jac_threads<128, JAC_LPP_SINGLE>()), 0, st, p);
      break;
  }
  return hipGetLastError();
}

namespace {
template <int LPP>
hipError_t launch_jacobi_batched_lpp(int variant, const JacobiParams* ps, const BlockMap* bm, dim3 grid,
                                     hipStream_t st) {
  switch (variant) {
    case 32: hipLaunchKernelGGL((jacobi_batched<32, LPP>), grid, dim3(jac_threads<32, LPP>()), 0, st, ps, bm); break;
    case 64: hipLaunchKernelGGL((jacobi_batched<64, LPP>), grid, dim3(jac_threads<64, LPP>()), 0, st, ps, bm); break;
    case 80: hipLaunchKernelGGL((jacobi_batched<80, LPP>), grid, dim3(jac_threads<80, LPP>()), 0, st, ps, bm); break;
    case 96: hipLaunchKernelGGL((jacobi_batched<96, LPP>), grid, dim3(jac_threads<96, LPP>()), 0, st, ps, bm); break;
    case 128:
      hipLaunchKernelGGL((jacobi_batched<128, LPP>), grid, dim3(jac_threads<128, LPP>()), 0, st, ps, bm);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_jacobi_batched(int variant, const JacobiParams* ps, const BlockMap* bm, int64_t nblocks,
                                 hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)nblocks);
  if (nblocks < JAC_BATCH_WIDE) return launch_jacobi_batched_lpp<JAC_LPP_SINGLE>(variant, ps, bm, grid, st);
  return launch_jacobi_batched_lpp<JAC_LPP_BATCH>(variant, ps, bm, grid, st);
}

}  // namespace rsvd
