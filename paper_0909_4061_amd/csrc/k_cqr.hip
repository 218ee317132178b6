// CholeskyQR building blocks: the orthonormalization "Y = QR" that follows
// every application of A or A* in Stage A (Algorithm 4.1 step 3, Algorithm 4.4
// steps 2, 4, 5; Section 4.1 allows any stable QR).  One CholeskyQR pass is
//   W = Y^T Y (FP64),  W = R^T R (Cholesky),  Q = Y R^-1,
// and CholeskyQR2 repeats it once on Q.  The host chains these kernels:
//
//   gram_partial : one workgroup per 64 rows.  Loads the rows of Y -- either
//                  summing the split-K partial products of the GEMM that made
//                  Y (in a fixed order) and storing Y, or reading a stored Y --
//                  and forms the 64-row block Gram Y_b^T Y_b with FP64 MFMA
//                  (FP32 entries are exact in FP64, so the products are exact).
//                  Only the upper 16x16 tiles are computed.
//   gram_reduce  : sums the block Grams in a fixed order (deterministic).
//   chol         : one workgroup of 512 threads.  Blocked (by 16) Cholesky
//                  of W in LDS, then the inverse R^-1 blockwise, a few
//                  barriers per block instead of per column.
//                  A pivot that is not safely positive restarts the
//                  factorization on W + sI (shifted CholeskyQR) and raises a
//                  flag; the host then runs a third pass.
//   trmm_upper   : R = R2 R1 for the combined factor.
#include <float.h>

#include "common.hpp"

namespace rsvd {

namespace {

template <typename T>
__device__ __forceinline__ void gram_partial_body(const GramParams& p, const int bid) {
  constexpr int RB = GRAM_ROWS;
  constexpr int YLD = 128 + 1;
  __shared__ T Ys[RB * YLD];
  if (p.gate && *p.gate == 0) return;
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)bid * RB;
  const int l = p.l, Lg = p.Lg;

  // Stage the rows (zero beyond l columns / beyond the last row).  Thread
  // tid covers column tid % 128 of rows tid / 128 + 2 it; every load of the
  // stage is issued before the first is used.
  constexpr int ITER = RB * 128 / 256;
  T vals[ITER];
#pragma unroll
  for (int it = 0; it < ITER; ++it) vals[it] = (T)0;
  const int c = tid & 127;
  const int rbase = tid >> 7;
  if (p.mode == GRAM_FROM_PART) {
    const T* __restrict__ part = (const T*)p.part;
    for (int s = 0; s < p.S; ++s) {
      const T* __restrict__ ps = part + (int64_t)s * p.rows * p.Lp;
#pragma unroll
      for (int it = 0; it < ITER; ++it) {
        const int64_t row = row0 + rbase + 2 * it;
        if (row < p.rows && c < l) vals[it] += ps[row * p.Lp + c];
      }
    }
    T* __restrict__ yout = (T*)p.yout;
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int64_t row = row0 + rbase + 2 * it;
      if (row < p.rows && c < l) yout[row * p.ldy + c] = vals[it];
    }
  } else {
    const T* __restrict__ yin = (const T*)p.yin;
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int64_t row = row0 + rbase + 2 * it;
      if (row < p.rows && c < l) vals[it] = yin[row * p.ldy + c];
    }
  }
  if (c < Lg) {
#pragma unroll
    for (int it = 0; it < ITER; ++it) Ys[(rbase + 2 * it) * YLD + c] = vals[it];
  }
  if (!p.do_gram) return;
  __syncthreads();

  // Upper 16x16 tiles of Y_b^T Y_b.  v_mfma_f64_16x16x4f64: A[i = lane%16][k =
  // lane/16] = Y[k][16 ti + i], B[k = lane/16][j = lane%16] = Y[k][16 tj + j];
  // result register e of lane holds G[16 ti + 4 e + lane/16][16 tj + lane%16].
  const int lane = tid & 63, wave = tid >> 6;
  const int nt = Lg / 16;
  const int ntiles = nt * (nt + 1) / 2;
  double* gout = p.gpart + (int64_t)bid * Lg * Lg;
  for (int tile = wave; tile < ntiles; tile += 4) {
    int ti = 0, rem = tile;
    while (rem >= nt - ti) {
      rem -= nt - ti;
      ++ti;
    }
    const int tj = ti + rem;
    f64x4 acc = f64x4{};
#pragma unroll 4
    for (int ks = 0; ks < RB / 4; ++ks) {
      const int kr = 4 * ks + (lane >> 4);
      const double a = (double)Ys[kr * YLD + 16 * ti + (lane & 15)];
      const double b = (double)Ys[kr * YLD + 16 * tj + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      gout[(int64_t)(16 * ti + 4 * e + (lane >> 4)) * Lg + 16 * tj + (lane & 15)] = acc[e];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void gram_partial_kernel(const GramParams p) { gram_partial_body<T>(p, blockIdx.x); }

template <typename T>
__global__ __launch_bounds__(256) void gram_partial_batched(const GramParams* __restrict__ ps, const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  gram_partial_body<T>(ps[b.item], b.local);
}

// Four threads per Gram entry, each summing every fourth block Gram; the four
// sums are combined in a fixed order.
__device__ __forceinline__ void gram_reduce_body(const GramReduceParams& p, const int bid) {
  __shared__ double red[4][64];
  if (p.gate && *p.gate == 0) return;
  const int tid = threadIdx.x;
  const int q = tid >> 6;
  const int64_t e = (int64_t)bid * 64 + (tid & 63);
  const int64_t LL = (int64_t)p.Lg * p.Lg;
  const bool live = e < LL && (e % p.Lg) >= (e / p.Lg);  // upper triangle only
  double acc = 0.0;
  if (live)
    for (int64_t b = q; b < p.nblk; b += 4) acc += p.gpart[b * LL + e];
  red[q][tid & 63] = acc;
  __syncthreads();
  if (q == 0 && e < LL) {
    const double v = live ? ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid] : 0.0;
    p.G[e] = v;
    if (live && !isfinite(v)) atomicOr(p.status, (int32_t)RSVD_FLAG_NONFINITE);
  }
}

__global__ __launch_bounds__(256) void gram_reduce_kernel(const GramReduceParams p) { gram_reduce_body(p, blockIdx.x); }

__global__ __launch_bounds__(256) void gram_reduce_batched(const GramReduceParams* __restrict__ ps,
                                                           const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  gram_reduce_body(ps[b.item], b.local);
}

// Cholesky factor R (W = R^T R, R upper triangular, positive diagonal) and its
// inverse X = R^-1, blocked by 16 for one workgroup of 512 threads.  W, then
// R, lives in the upper triangle of an LDS matrix; X^T is built in the strict
// lower triangle (X is upper triangular) and 1 / R_ii in a vector.
//
// Factorization, per block column [k0, k1):
//   1. one wave factors the panel (rows k0..k1-1) in registers, right-looking:
//      lanes 0..15 hold the diagonal block's columns, lanes 16..63 three
//      columns each of the block row (R_kj = R_kk^-T W_kj); the pivots and
//      the rows of R_kk are broadcast with readlane;
//   2. the trailing matrix is updated, W_ij -= R_ki^T R_kj for k1 <= i <= j:
//      one column per lane, eight rows per wave, the rows of R_k read as LDS
//      broadcasts.
// Inverse by doubling: every 16 x 16 diagonal block inverted at once (one
// column per lane), then for s = 16, 32, 64 each aligned pair of inverted
// blocks [A C] is joined, X_AC = -X_AA (R_AC X_CC), again one column per lane
// and eight rows per wave.
// A pivot that is not positive (or not finite) restarts the factorization on
// W + s I with the shifted-CholeskyQR shift; a second failure (non-finite
// input) returns identity factors and raises RSVD_FLAG_NONFINITE.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// 1/sqrt(x) from the hardware estimate and two Newton steps (x > 0, finite).
__device__ __forceinline__ double rsq_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

__device__ __forceinline__ void chol_body(const CholParams& p, const int bid) {
  (void)bid;  // one workgroup per factorization
  constexpr int NT = 512, NW = NT / 64, B = 16, LDC = 129;  // odd stride: column walks hit distinct banks
  constexpr int RG = 8;                                      // rows per wave in the matrix phases
  __shared__ double M[128 * LDC];
  __shared__ double rinv_d[128];  // 1 / R_ii (0 past l)
  __shared__ int bad_s;
  if (p.gate && *p.gate == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l = p.l, Lg = p.Lg;
  const int lp = (l + B - 1) & ~(B - 1);  // rows and columns past l up to lp hold zeros
  const int tc = tid & 127, tr = tid >> 7;  // 4 x 128 thread grid for whole-matrix loops
  const double eps = DBL_EPSILON;
  double thresh = 0.0, trace = 0.0;

  bool ok = false;
  for (int attempt = 0; attempt < 2 && !ok; ++attempt) {
    // Shifted CholeskyQR: s = 11 (rows l + l (l + 1)) u ||Y||_F^2 with u the FP64 unit roundoff.
    const double shift =
        attempt == 0 ? 0.0 : 11.0 * ((double)p.rows * l + (double)l * (l + 1)) * (0.5 * eps) * trace;
    for (int a0 = tr; a0 < lp; a0 += 4 * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int a = a0 + 4 * u;
        v[u] = (a < l && tc < l && tc >= a) ? p.G[(int64_t)a * Lg + tc] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int a = a0 + 4 * u;
        if (a < lp && tc < lp) M[a * LDC + tc] = v[u] + (a == tc && a < l ? shift : 0.0);
      }
    }
    if (tid < 128) rinv_d[tid] = 0.0;
    __syncthreads();
    if (attempt == 0) {
      // max diagonal (breakdown threshold) and trace (shift) of W, every wave for itself
      const double d0 = lane < l ? p.G[(int64_t)lane * (Lg + 1)] : 0.0;
      const double d1 = lane + 64 < l ? p.G[(int64_t)(lane + 64) * (Lg + 1)] : 0.0;
      double mx = fmax(d0, d1), trs = d0 + d1;
      for (int off = 32; off > 0; off >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, off, 64));
        trs += __shfl_xor(trs, off, 64);
      }
      thresh = (double)l * 16.0 * eps * mx;
      trace = trs;
    }
    ok = true;
    for (int k0 = 0; k0 < l; k0 += B) {
      const int k1 = min(k0 + B, l), bk = k1 - k0;
      // 1. panel by wave 0.  Past the diagonal block the block is full (bk == B):
      //    only the last one is partial, and it has no block row.
      if (wave == 0) {
        int col[3];
        bool has[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          col[m] = lane < B ? k0 + lane : k1 + (lane - B) + 48 * m;
          has[m] = lane < B ? (m == 0 && lane < bk) : col[m] < l;
        }
        double x[3][B];
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
          for (int i = 0; i < B; ++i)
            x[m][i] = (has[m] && (lane >= B || i <= lane)) ? M[(k0 + i) * LDC + col[m]] : 0.0;
        int bad = 0;
#pragma unroll
        for (int j = 0; j < B; ++j) {
          if (j < bk && !bad) {  // uniform across the wave
            const double djj = readlane_f64(x[0][j], j);
            if (!(djj > thresh) || !isfinite(djj)) {
              bad = 1;
            } else {
              const double rinv = rsq_refined(djj);
              double rjj = djj * rinv;
              rjj = fma(0.5 * rinv, fma(-rjj, rjj, djj), rjj);
#pragma unroll
              for (int m = 0; m < 3; ++m) x[m][j] *= rinv;  // row j of R (zeros stay zeros)
              if (lane == j) {
                x[0][j] = rjj;
                rinv_d[k0 + j] = rinv;
              }
#pragma unroll
              for (int i = j + 1; i < B; ++i) {
                const double rji = readlane_f64(x[0][j], i);  // R[j][i]
#pragma unroll
                for (int m = 0; m < 3; ++m) x[m][i] = fma(-rji, x[m][j], x[m][i]);
              }
            }
          }
        }
        if (!bad) {
#pragma unroll
          for (int m = 0; m < 3; ++m)
            if (has[m])
#pragma unroll
              for (int i = 0; i < B; ++i)
                if (lane >= B || i <= lane) M[(k0 + i) * LDC + col[m]] = x[m][i];
        }
        if (lane == 0) bad_s = bad;
      }
      __syncthreads();
      if (bad_s) {
        ok = false;
        break;
      }
      // 2. trailing update: item = (64-column chunk, 8-row group) per wave
      const int nt = l - k1;
      if (nt > 0) {
        const int nrg = (nt + RG - 1) / RG, items = ((nt + 63) / 64) * nrg;
        for (int it = wave; it < items; it += NW) {
          const int cc = it / nrg, rg = it - cc * nrg;
          const int i0 = k1 + RG * rg, cbase = k1 + 64 * cc;
          if (i0 > cbase + 63) continue;  // below the diagonal (uniform)
          const int c = cbase + lane, cl = min(c, lp - 1);
          double acc[RG] = {};
#pragma unroll 4
          for (int t = 0; t < B; ++t) {
            const double* row = M + (k0 + t) * LDC;
            const double bv = row[cl];
#pragma unroll
            for (int i = 0; i < RG; ++i) acc[i] = fma(row[i0 + i], bv, acc[i]);
          }
          if (c < l)
#pragma unroll
            for (int i = 0; i < RG; ++i)
              if (i0 + i <= c) M[(i0 + i) * LDC + c] -= acc[i];
        }
      }
      __syncthreads();
    }
    if (!ok && attempt == 0 && tid == 0) {
      atomicOr(p.status, (int32_t)RSVD_FLAG_SHIFTED);
      if (p.shifted) *p.shifted = 1;
    }
    __syncthreads();  // every thread has read bad_s before the next attempt rewrites M
  }
  if (!ok) {
    // Shifted factorization failed as well (non-finite input): identity factors.
    if (tid == 0) atomicOr(p.status, (int32_t)RSVD_FLAG_NONFINITE);
    for (int a = tr; a < l; a += 4) {
      if (tc >= l) break;
      const int64_t idx = (int64_t)a * l + tc;
      const double v = a == tc ? 1.0 : 0.0;
      if (p.R) p.R[idx] = v;
      if (p.Rinv) p.Rinv[idx] = v;
      if (p.RinvT) {
        if (p.dtype == RSVD_F64) ((double*)p.RinvT)[idx] = v;
        else ((float*)p.RinvT)[idx] = (float)v;
      }
    }
    return;
  }
  if (p.R && tc < l)
    for (int a = tr; a < l; a += 4) p.R[(int64_t)a * l + tc] = tc >= a ? M[a * LDC + tc] : 0.0;
  if (!p.Rinv && !p.RinvT) return;

  // Inverse.  X[r][c] (r < c) is kept at M[c * LDC + r], X[c][c] in rinv_d.
  const int nb = lp / B;
  // diagonal blocks, one wave each: lane c solves R_bb x = e_c, right-looking from the bottom
  for (int b = wave; b < nb; b += NW) {
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
  // Joining pairs: A = [a0, a1) (full, s rows), C = [a1, ce) (s columns, the last
  // pair possibly fewer).  Item = (pair, 8-row group of A) per wave, lane = column of C;
  // npair * s / 8 = 8 items per level for l <= 128.
  for (int s = B; s < l; s *= 2) {
    const int npair = (l - s + 2 * s - 1) / (2 * s);
    const int nrg = s / RG, items = npair * nrg;
    for (int it0 = 0; it0 < items; it0 += NW) {
      const int it = it0 + wave;
      const int pair = it / nrg, rg = it - pair * nrg;
      const int a1 = 2 * s * pair + s, ce = min(a1 + s, l);
      const int r0 = a1 - s + RG * rg, c = a1 + lane;
      const bool work = it < items && lane < s && c < ce;
      double acc[RG] = {};
      // T = R_AC X_CC: T[r][c] = sum_{t = a1..c} R[r][t] X[t][c]
      if (work) {
        for (int t = a1; t < c; ++t) {
          const double bv = M[c * LDC + t];
#pragma unroll
          for (int i = 0; i < RG; ++i) acc[i] = fma(M[(r0 + i) * LDC + t], bv, acc[i]);
        }
        const double bv = rinv_d[c];
#pragma unroll
        for (int i = 0; i < RG; ++i) {
          acc[i] = fma(M[(r0 + i) * LDC + c], bv, acc[i]);
          M[c * LDC + r0 + i] = acc[i];
        }
      }
      __syncthreads();
      // X_AC = -X_AA T: X[r][c] = -sum_{u = r..a1-1} X[r][u] T[u][c]
      if (work) {
#pragma unroll
        for (int i = 0; i < RG; ++i) acc[i] = 0.0;
#pragma unroll
        for (int uu = 0; uu < RG; ++uu) {
          const int u = r0 + uu;
          const double bv = M[c * LDC + u];
#pragma unroll
          for (int i = 0; i < RG; ++i) {
            const double av = uu > i ? M[u * LDC + r0 + i] : (uu == i ? rinv_d[u] : 0.0);
            acc[i] = fma(av, bv, acc[i]);
          }
        }
        for (int u = r0 + RG; u < a1; ++u) {
          const double bv = M[c * LDC + u];
#pragma unroll
          for (int i = 0; i < RG; ++i) acc[i] = fma(M[u * LDC + r0 + i], bv, acc[i]);
        }
      }
      __syncthreads();
      if (work)
#pragma unroll
        for (int i = 0; i < RG; ++i) M[c * LDC + r0 + i] = -acc[i];
      __syncthreads();
    }
  }
  if (tc < l)
    for (int a = tr; a < l; a += 4) {
      const int64_t idx = (int64_t)a * l + tc;
      const double v = tc > a ? M[tc * LDC + a] : (tc == a ? rinv_d[a] : 0.0);
      if (p.Rinv) p.Rinv[idx] = v;
      if (p.RinvT) {
        if (p.dtype == RSVD_F64) ((double*)p.RinvT)[idx] = v;
        else ((float*)p.RinvT)[idx] = (float)v;
      }
    }
}

__global__ __launch_bounds__(512) void chol_kernel(const CholParams p) { chol_body(p, blockIdx.x); }

__global__ __launch_bounds__(512) void chol_batched(const CholParams* __restrict__ ps, const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  chol_body(ps[b.item], b.local);
}

__device__ __forceinline__ void trmm_body(const TrmmParams& p, const int bid) {
  if (p.gate && *p.gate == 0) return;
  const int l = p.l;
  const int64_t idx = (int64_t)bid * 256 + threadIdx.x;
  if (idx >= (int64_t)l * l) return;
  const int i = (int)(idx / l), j = (int)(idx - (int64_t)i * l);
  double acc = 0.0;
  for (int t = i; t <= j; ++t) acc += p.R2[(int64_t)i * l + t] * p.R1[(int64_t)t * l + j];
  p.R[idx] = acc;
}

__global__ __launch_bounds__(256) void trmm_upper_kernel(const TrmmParams p) { trmm_body(p, blockIdx.x); }

__global__ __launch_bounds__(256) void trmm_batched(const TrmmParams* __restrict__ ps, const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  trmm_body(ps[b.item], b.local);
}

__device__ __forceinline__ void copy_body(const CopyParams& p, const int bid) {
  if (p.gate && *p.gate == 0) return;
  const int64_t i = (int64_t)bid * 256 + threadIdx.x;
  if (i < p.count) p.dst[i] = p.src[i];
}

__global__ __launch_bounds__(256) void copy_f64_kernel(const CopyParams p) { copy_body(p, blockIdx.x); }

__global__ __launch_bounds__(256) void copy_batched(const CopyParams* __restrict__ ps, const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  copy_body(ps[b.item], b.local);
}

}  // namespace

int64_t trmm_blocks(const TrmmParams& p) { return ((int64_t)p.l * p.l + 255) / 256; }

int64_t copy_blocks(const CopyParams& p) { return (p.count + 255) / 256; }

hipError_t launch_copy_f64(const double* src, double* dst, int64_t count, const int32_t* gate, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const CopyParams p{src, dst, count, gate};
  hipLaunchKernelGGL(copy_f64_kernel, dim3((unsigned)copy_blocks(p)), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_trmm_batched(const TrmmParams* ps, const BlockMap* bm, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(trmm_batched, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
  return hipGetLastError();
}

hipError_t launch_copy_batched(const CopyParams* ps, const BlockMap* bm, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_batched, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
  return hipGetLastError();
}

hipError_t launch_gram_partial(int dtype, const GramParams& p, hipStream_t st) {
  if (p.rows <= 0) return hipSuccess;
  if (p.l > 128 || p.Lg % 16 != 0 || p.Lg < p.l) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((p.rows + GRAM_ROWS - 1) / GRAM_ROWS));
  if (dtype == RSVD_F64)
    hipLaunchKernelGGL(gram_partial_kernel<double>, grid, dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(gram_partial_kernel<float>, grid, dim3(256), 0, st, p);
  return hipGetLastError();
}

int64_t gram_partial_blocks(const GramParams& p) { return (p.rows + GRAM_ROWS - 1) / GRAM_ROWS; }

int64_t gram_reduce_blocks(const GramReduceParams& p) { return ((int64_t)p.Lg * p.Lg + 63) / 64; }

hipError_t launch_gram_reduce(const double* gpart, int64_t nblk, int32_t Lg, double* G, int32_t* status,
                              const int32_t* gate, hipStream_t st) {
  const GramReduceParams p{gpart, nblk, Lg, G, status, gate};
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)gram_reduce_blocks(p)), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_gram_partial_batched(int dtype, const GramParams* ps, const BlockMap* bm, int64_t nblocks,
                                       hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (dtype == RSVD_F64)
    hipLaunchKernelGGL(gram_partial_batched<double>, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
  else
    hipLaunchKernelGGL(gram_partial_batched<float>, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
  return hipGetLastError();
}

hipError_t launch_gram_reduce_batched(const GramReduceParams* ps, const BlockMap* bm, int64_t nblocks,
                                      hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(gram_reduce_batched, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
  return hipGetLastError();
}

hipError_t launch_chol_batched(const CholParams* ps, const BlockMap* bm, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(chol_batched, dim3((unsigned)nblocks), dim3(512), 0, st, ps, bm);
  return hipGetLastError();
}

hipError_t launch_chol(const CholParams& p, hipStream_t st) {
  if (p.l > 128 || p.l < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(512), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_trmm_upper(const double* R2, const double* R1, double* R, int32_t l, const int32_t* gate,
                             hipStream_t st) {
  const TrmmParams p{R2, R1, R, l, gate};
  hipLaunchKernelGGL(trmm_upper_kernel, dim3((unsigned)trmm_blocks(p)), dim3(256), 0, st, p);
  return hipGetLastError();
}

}  // namespace rsvd
