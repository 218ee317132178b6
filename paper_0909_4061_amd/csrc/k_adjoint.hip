// Pieces of the adjoint (reverse-mode derivative) of the fixed-Omega randomized
// SVD that are not products with A: the l x l algebra of the SVD and QR
// adjoints, in FP64, and a strided copy / transpose / type cast.
//
// SVD of the small matrix, B = U~ S V~^T (l x n, l <= n, full rank), seen as
// the tall factorization B^T = V~ S U~^T.  With the incoming adjoints gS (k),
// gU~ = [Q^T gU, 0] (l x l) and gV~ = [gV, 0] (n x l) (the truncation to k
// triplets pads them with zeros), the adjoint of B^T is
//   gB^T = V~ [ (F o (V~^T gV~ - gV~^T V~)) S + diag(gS) + S (F o (U~^T gU~ - gU~^T U~)) ] U~^T
//          + (I - V~ V~^T) gV~ S^-1 U~^T,
// F_ij = 1 / (s_j^2 - s_i^2) (i != j), F_ii = 0 -- the standard thin-SVD
// derivative.  With V~ = B^T U~ S^-1 this becomes
//   gB^T = B^T M1 + gV M2,  M1 = U~ S^-1 (C - P1 S^-1) U~^T,  M2 = S_k^-1 U~_k^T,
// where C is the bracket and P1 = V~^T gV~ = S^-1 U~^T (B gV).
// svd_adj_coef_kernel forms Z = S^-1 (C - P1 S^-1) entry by entry; two FP64
// products give M1 = U~ Z U~^T.
//
// QR, Y = Q R with R upper triangular, positive diagonal, and only Q used
// downstream: gY = (gQ + Q sym(-gQ^T Q)) R^-T, where sym(X) copies the lower
// triangle of X (diagonal included) onto the upper one.
#include "common.hpp"

namespace rsvd {

namespace {

template <typename T>
__device__ __forceinline__ double ld_as_f64(const void* p, int64_t i) {
  return (double)static_cast<const T*>(p)[i];
}

__device__ __forceinline__ double ld_elem(const void* p, int dtype, int64_t i) {
  return dtype == RSVD_F64 ? ld_as_f64<double>(p, i) : ld_as_f64<float>(p, i);
}

__device__ __forceinline__ void svd_adj_coef_body(const SvdAdjParams& p, const int bid) {
  const int l = p.l, k = p.k;
  const int64_t e = (int64_t)bid * 256 + threadIdx.x;
  if (e >= (int64_t)l * l) return;
  const int i = (int)(e / l), j = (int)(e - (int64_t)i * l);
  const double si = p.sig[i], sj = p.sig[j];
  // P1_ab = (1/s_a) sum_r U~_ra T1_rb  (b < k), P2_ab = sum_r U~_ra T2_rb  (b < k)
  double d1ij = 0.0, d1ji = 0.0, d2ij = 0.0, d2ji = 0.0;
  for (int r = 0; r < l; ++r) {
    const double uri = p.Uh[(int64_t)r * l + i], urj = p.Uh[(int64_t)r * l + j];
    if (j < k) {
      d1ij += uri * ld_elem(p.T1, p.dtype, (int64_t)r * k + j);
      d2ij += uri * ld_elem(p.T2, p.dtype, (int64_t)r * k + j);
    }
    if (i < k) {
      d1ji += urj * ld_elem(p.T1, p.dtype, (int64_t)r * k + i);
      d2ji += urj * ld_elem(p.T2, p.dtype, (int64_t)r * k + i);
    }
  }
  const double p1ij = d1ij / si, p1ji = d1ji / sj;
  const double F = i != j ? 1.0 / (sj * sj - si * si) : 0.0;
  double c = F * (p1ij - p1ji) * sj + si * F * (d2ij - d2ji);
  if (i == j && i < k) c += ld_elem(p.gS, p.dtype, i);
  p.Z[e] = (c - p1ij / sj) / si;
  if (i < k) {
    // row i of U~_k^T and of S_k^-1 U~_k^T (column j)
    const double u = p.Uh[(int64_t)j * l + i];
    p.Ukt[(int64_t)i * l + j] = u;
    p.M2[(int64_t)i * l + j] = u / si;
  }
}

__global__ __launch_bounds__(256) void svd_adj_coef_kernel(const SvdAdjParams p) { svd_adj_coef_body(p, blockIdx.x); }

__global__ __launch_bounds__(256) void svd_adj_coef_batched(const SvdAdjParams* __restrict__ ps,
                                                            const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  svd_adj_coef_body(ps[b.item], b.local);
}

// S_ij = -M_{min(i,j), max(i,j)}: sym(-M^T) for M = Q^T gQ.
__device__ __forceinline__ void qr_adj_sym_body(const QrSymParams& p, const int bid) {
  const int l = p.l;
  const int64_t e = (int64_t)bid * 256 + threadIdx.x;
  if (e >= (int64_t)l * l) return;
  const int i = (int)(e / l), j = (int)(e - (int64_t)i * l);
  const int a = min(i, j), b = max(i, j);
  p.S[e] = -ld_elem(p.M, p.dtype, (int64_t)a * l + b);
}

__global__ __launch_bounds__(256) void qr_adj_sym_kernel(const QrSymParams p) { qr_adj_sym_body(p, blockIdx.x); }

__global__ __launch_bounds__(256) void qr_adj_sym_batched(const QrSymParams* __restrict__ ps,
                                                          const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  qr_adj_sym_body(ps[b.item], b.local);
}

// Rinv = R^-1 for upper triangular R (l x l <= 128 x 128), one workgroup of
// 256 threads, R in LDS.  X = R^-1 by doubling: every 16 x 16 diagonal block
// is inverted at once (one wave per block, lane c solving R_bb x = e_c from the
// bottom), then for s = 16, 32, 64 each aligned pair of inverted blocks [A C]
// is joined, X_AC = -X_AA (R_AC X_CC): an item is (pair, 8 rows of A) per
// wave, one column of C per lane.  X[r][c] (r < c) is kept at M[c * LDC + r],
// X[c][c] = 1 / R_cc in a vector; rows and columns past l up to a multiple of
// 16 are zeros.
__device__ __forceinline__ void tri_inv_upper_body(const TriInvParams& p) {
  const double* __restrict__ R = p.R;
  double* __restrict__ Rinv = p.Rinv;
  const int l = p.l;
  constexpr int NW = 4, B = 16, RG = 8, LDC = 129;  // odd stride: column walks hit distinct banks
  __shared__ double M[128 * LDC];
  __shared__ double rinv_d[128];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lp = (l + B - 1) & ~(B - 1);
  const int tc = tid & 127, tr = tid >> 7;  // 2 x 128 thread grid for whole-matrix loops
  if (tc < lp)
    for (int a = tr; a < lp; a += 2) M[a * LDC + tc] = (a < l && tc < l && tc >= a) ? R[(int64_t)a * l + tc] : 0.0;
  if (tid < 128) rinv_d[tid] = tid < l ? 1.0 / R[(int64_t)tid * l + tid] : 0.0;
  __syncthreads();
  // diagonal blocks
  for (int b = wave; b < lp / B; b += NW) {
    const int b0 = b * B;
    double acc[B], x[B];
#pragma unroll
    for (int i = 0; i < B; ++i) acc[i] = 0.0;
#pragma unroll
    for (int t = B - 1; t >= 0; --t) {
      const double rt = rinv_d[b0 + t];
      x[t] = t == lane ? rt : (t < lane ? -acc[t] * rt : 0.0);
#pragma unroll
      for (int i = 0; i < t; ++i) acc[i] = fma(M[(b0 + i) * LDC + b0 + t], x[t], acc[i]);
    }
    if (lane < B && b0 + lane < l) {
#pragma unroll
      for (int i = 0; i < B; ++i)
        if (i < lane) M[(b0 + lane) * LDC + b0 + i] = x[i];
    }
  }
  __syncthreads();
  // joining pairs: A = [a1 - s, a1) (full), C = [a1, ce) (s columns, the last pair
  // possibly fewer); npair * s / 8 <= 8 items per level for l <= 128, two per wave.
  // Every T of a level is formed before any X_AC, which reads T rows of the other
  // items of its pair.
  constexpr int IPW = 2;  // items per wave
  for (int s = B; s < l; s *= 2) {
    const int npair = (l - s + 2 * s - 1) / (2 * s);
    const int nrg = s / RG, items = npair * nrg;
    int r0[IPW], c[IPW], a1[IPW];
    bool work[IPW];
#pragma unroll
    for (int j = 0; j < IPW; ++j) {
      const int it = wave + NW * j;
      const int pair = it / nrg, rg = it - pair * nrg;
      a1[j] = 2 * s * pair + s;
      const int ce = min(a1[j] + s, l);
      r0[j] = a1[j] - s + RG * rg;
      c[j] = a1[j] + lane;
      work[j] = it < items && lane < s && c[j] < ce;
    }
    // T = R_AC X_CC: T[r][c] = sum_{t = a1..c} R[r][t] X[t][c], stored in the X_AC slots
#pragma unroll
    for (int j = 0; j < IPW; ++j) {
      if (work[j]) {
        double acc[RG] = {};
        for (int t = a1[j]; t < c[j]; ++t) {
          const double bv = M[c[j] * LDC + t];
#pragma unroll
          for (int i = 0; i < RG; ++i) acc[i] = fma(M[(r0[j] + i) * LDC + t], bv, acc[i]);
        }
        const double bv = rinv_d[c[j]];
#pragma unroll
        for (int i = 0; i < RG; ++i) {
          acc[i] = fma(M[(r0[j] + i) * LDC + c[j]], bv, acc[i]);
          M[c[j] * LDC + r0[j] + i] = acc[i];
        }
      }
    }
    __syncthreads();
    // X_AC = -X_AA T: X[r][c] = -sum_{u = r..a1-1} X[r][u] T[u][c]
    double accx[IPW][RG];
#pragma unroll
    for (int j = 0; j < IPW; ++j) {
#pragma unroll
      for (int i = 0; i < RG; ++i) accx[j][i] = 0.0;
      if (work[j]) {
#pragma unroll
        for (int uu = 0; uu < RG; ++uu) {
          const int u = r0[j] + uu;
          const double bv = M[c[j] * LDC + u];
#pragma unroll
          for (int i = 0; i < RG; ++i) {
            const double av = uu > i ? M[u * LDC + r0[j] + i] : (uu == i ? rinv_d[u] : 0.0);
            accx[j][i] = fma(av, bv, accx[j][i]);
          }
        }
        for (int u = r0[j] + RG; u < a1[j]; ++u) {
          const double bv = M[c[j] * LDC + u];
#pragma unroll
          for (int i = 0; i < RG; ++i) accx[j][i] = fma(M[u * LDC + r0[j] + i], bv, accx[j][i]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPW; ++j)
      if (work[j])
#pragma unroll
        for (int i = 0; i < RG; ++i) M[c[j] * LDC + r0[j] + i] = -accx[j][i];
    __syncthreads();
  }
  if (tc < l)
    for (int a = tr; a < l; a += 2)
      Rinv[(int64_t)a * l + tc] = tc > a ? M[tc * LDC + a] : (tc == a ? rinv_d[a] : 0.0);
}

__global__ __launch_bounds__(256) void tri_inv_upper_kernel(const TriInvParams p) { tri_inv_upper_body(p); }

__global__ __launch_bounds__(256) void tri_inv_upper_batched(const TriInvParams* __restrict__ ps,
                                                             const BlockMap* __restrict__ bm) {
  tri_inv_upper_body(ps[bm[blockIdx.x].item]);
}

// dst (rows x cols, or cols x rows when transposed) <- src (rows x cols),
// with a cast between FP32 and FP64.  32 x 32 tiles through LDS.
__device__ __forceinline__ void copy2d_body(const Copy2dParams& p, const int bid) {
  __shared__ double tile[32][33];
  const int gx = (int)((p.cols + 31) / 32);  // tiles across the source columns
  const int64_t r0 = (int64_t)(bid / gx) * 32, c0 = (int64_t)(bid % gx) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int rr = ty; rr < 32; rr += 8) {
    const int64_t r = r0 + rr, c = c0 + tx;
    if (r < p.rows && c < p.cols) tile[rr][tx] = ld_elem(p.src, p.src_dtype, r * p.lds + c);
  }
  __syncthreads();
  for (int rr = ty; rr < 32; rr += 8) {
    int64_t dr, dc;
    double v;
    if (p.trans) {  // dst[c][r] = src[r][c]: walk dst rows = source columns
      dc = r0 + tx;
      dr = c0 + rr;
      if (dc >= p.rows || dr >= p.cols) continue;
      v = tile[tx][rr];
    } else {
      dr = r0 + rr;
      dc = c0 + tx;
      if (dr >= p.rows || dc >= p.cols) continue;
      v = tile[rr][tx];
    }
    const int64_t o = dr * p.ldd + dc;
    if (p.negate) v = -v;
    if (p.dst_dtype == RSVD_F64)
      static_cast<double*>(p.dst)[o] = v;
    else
      static_cast<float*>(p.dst)[o] = (float)v;
  }
}

__global__ __launch_bounds__(256) void copy2d_kernel(const Copy2dParams p) { copy2d_body(p, blockIdx.x); }

__global__ __launch_bounds__(256) void copy2d_batched(const Copy2dParams* __restrict__ ps,
                                                      const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  copy2d_body(ps[b.item], b.local);
}

}  // namespace

int64_t svd_adj_coef_blocks(const SvdAdjParams& p) { return ((int64_t)p.l * p.l + 255) / 256; }
int64_t qr_adj_sym_blocks(const QrSymParams& p) { return ((int64_t)p.l * p.l + 255) / 256; }
int64_t copy2d_blocks(const Copy2dParams& p) {
  return p.rows <= 0 || p.cols <= 0 ? 0 : ((p.cols + 31) / 32) * ((p.rows + 31) / 32);
}
bool svd_adj_coef_ok(const SvdAdjParams& p) { return p.l >= 1 && p.l <= RSVD_MAX_L && p.k >= 1 && p.k <= p.l; }
bool tri_inv_ok(const TriInvParams& p) { return p.l >= 1 && p.l <= 128; }

hipError_t launch_svd_adj_coef(const SvdAdjParams& p, hipStream_t st) {
  if (!svd_adj_coef_ok(p)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(svd_adj_coef_kernel, dim3((unsigned)svd_adj_coef_blocks(p)), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_qr_adj_sym(const QrSymParams& p, hipStream_t st) {
  hipLaunchKernelGGL(qr_adj_sym_kernel, dim3((unsigned)qr_adj_sym_blocks(p)), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_tri_inv_upper(const TriInvParams& p, hipStream_t st) {
  if (!tri_inv_ok(p)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tri_inv_upper_kernel, dim3(1), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_copy2d(const Copy2dParams& p, hipStream_t st) {
  const int64_t nb = copy2d_blocks(p);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(copy2d_kernel, dim3((unsigned)nb), dim3(256), 0, st, p);
  return hipGetLastError();
}

// Batched launches (parameters checked when each problem was recorded).
hipError_t launch_svd_adj_coef_batched(const SvdAdjParams* ps, const BlockMap* bm, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(svd_adj_coef_batched, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
  return hipGetLastError();
}

hipError_t launch_qr_adj_sym_batched(const QrSymParams* ps, const BlockMap* bm, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(qr_adj_sym_batched, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
  return hipGetLastError();
}

hipError_t launch_tri_inv_upper_batched(const TriInvParams* ps, const BlockMap* bm, int64_t nblocks,
                                        hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(tri_inv_upper_batched, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
  return hipGetLastError();
}

hipError_t launch_copy2d_batched(const Copy2dParams* ps, const BlockMap* bm, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy2d_batched, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
  return hipGetLastError();
}

}  // namespace rsvd
