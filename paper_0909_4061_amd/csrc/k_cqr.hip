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
//   chol         : one workgroup.  Symmetric elimination of W with the same
//                  row operations applied to the identity, both l x l arrays
//                  held in registers (1024 threads, 4x4 entries each), one
//                  barrier per column: the eliminated W is D L^T and the
//                  accumulated operations are L^-1, which gives
//                  R = D^-1/2 (D L^T) and R^-1 = L^-T D^-1/2 at once.
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

// Cholesky with simultaneous inverse.  Thread (tr, tc) of a 32 x 32 grid owns
// the entries (a, c), a = tr + 32 ia, c = tc + 32 ib (ia, ib < 4), of two
// register tiles: U (the eliminated matrix; only c >= a is meaningful) and E
// (the accumulated row operations, E = L^-1, lower triangular with unit
// diagonal).  Step j subtracts f_a = U[j][a] / U[j][j] times the pivot row from
// every row a > j: U[a][c] -= f_a U[j][c] for c > j and E[a][c] -= f_a E[j][c]
// for c <= j (E[j][j] = 1).  The masks fold into the multipliers, so each
// element costs two FMAs; waves whose rows are all finished skip the update.
// At the end U = D L^T, hence R = D^-1/2 U and R^-1 = E^T D^-1/2.
__device__ __forceinline__ void chol_body(const CholParams& p, const int bid) {
  (void)bid;  // one workgroup per factorization
  constexpr int TLD = 129;
  __shared__ double rowbuf[2][128];
  __shared__ double diag[128];
  __shared__ double red[32];
  __shared__ double tbuf[128 * TLD];
  if (p.gate && *p.gate == 0) return;
  const int tid = threadIdx.x;
  const int tr = tid >> 5, tc = tid & 31;
  const int wave_row_max = (tid >> 6) * 2 + 1;  // largest tr in this wave
  const int l = p.l, Lg = p.Lg;

  // max diagonal and trace of W (for the breakdown threshold and the shift)
  double dmax = 0.0, trace = 0.0;
  {
    const double dv = (tid < l) ? p.G[(int64_t)tid * Lg + tid] : 0.0;
    double m = dv, t = dv;
    for (int off = 16; off > 0; off >>= 1) {
      m = fmax(m, __shfl_xor(m, off, 32));
      t += __shfl_xor(t, off, 32);
    }
    if (tid < 128 && (tid & 31) == 0) {
      red[tid >> 5] = m;
      red[4 + (tid >> 5)] = t;
    }
    __syncthreads();
    for (int i = 0; i < 4; ++i) {
      dmax = fmax(dmax, red[i]);
      trace += red[4 + i];
    }
  }
  const double eps = DBL_EPSILON;
  const double thresh = (double)l * 16.0 * eps * dmax;

  double U[4][4], E[4][4];
  bool ok = false;
  for (int attempt = 0; attempt < 2 && !ok; ++attempt) {
    // Shifted CholeskyQR: s = 11 (rows l + l (l + 1)) u ||Y||_F^2 with u the FP64 unit roundoff.
    const double shift =
        attempt == 0 ? 0.0 : 11.0 * ((double)p.rows * l + (double)l * (l + 1)) * (0.5 * eps) * trace;
#pragma unroll
    for (int ia = 0; ia < 4; ++ia) {
      const int a = tr + 32 * ia;
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) {
        const int c = tc + 32 * ib;
        double v = 0.0;
        if (a < l && c < l && c >= a) v = p.G[(int64_t)a * Lg + c] + (c == a ? shift : 0.0);
        U[ia][ib] = v;
        E[ia][ib] = 0.0;
      }
    }
    if (tr == 0) {
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) rowbuf[0][tc + 32 * ib] = U[0][ib];
    }
    ok = true;
    for (int j = 0; j < l; ++j) {
      const int buf = j & 1;
      __syncthreads();
      const double d = rowbuf[buf][j];
      double prow[4], pcol[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        prow[i] = rowbuf[buf][tr + 32 * i];
        pcol[i] = rowbuf[buf][tc + 32 * i];
      }
      if (!(d > thresh) || !isfinite(d)) {  // uniform: every thread reads the same d
        ok = false;
        break;
      }
      if (tid == 0) diag[j] = d;
      const double invd = 1.0 / d;
      double pu[4], pe[4];
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) {
        const int c = tc + 32 * ib;
        pu[ib] = c > j ? pcol[ib] : 0.0;
        pe[ib] = c < j ? pcol[ib] : (c == j ? 1.0 : 0.0);
      }
#pragma unroll
      for (int ia = 0; ia < 4; ++ia) {
        if (wave_row_max + 32 * ia <= j) continue;  // wave-uniform: no live row in this block
        const int a = tr + 32 * ia;
        const double f = (a > j && a < l) ? prow[ia] * invd : 0.0;
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
          U[ia][ib] -= f * pu[ib];
          E[ia][ib] -= f * pe[ib];
        }
      }
      // the owners of row j + 1 publish it: U part right of the diagonal, E part left
#pragma unroll
      for (int ia = 0; ia < 4; ++ia) {
        if (tr + 32 * ia == j + 1) {
#pragma unroll
          for (int ib = 0; ib < 4; ++ib) {
            const int c = tc + 32 * ib;
            rowbuf[buf ^ 1][c] = c >= j + 1 ? U[ia][ib] : E[ia][ib];
          }
        }
      }
    }
    __syncthreads();
    if (!ok && attempt == 0 && tid == 0) {
      atomicOr(p.status, (int32_t)RSVD_FLAG_SHIFTED);
      if (p.shifted) *p.shifted = 1;
    }
  }
  if (!ok) {
    // Shifted factorization failed as well (non-finite input): identity factors.
    if (tid == 0) atomicOr(p.status, (int32_t)RSVD_FLAG_NONFINITE);
    for (int idx = tid; idx < l * l; idx += 1024) {
      const int a = idx / l, c = idx - a * l;
      const double v = a == c ? 1.0 : 0.0;
      if (p.R) p.R[idx] = v;
      if (p.Rinv) p.Rinv[idx] = v;
      if (p.RinvT) {
        if (p.dtype == RSVD_F64) ((double*)p.RinvT)[idx] = v;
        else ((float*)p.RinvT)[idx] = (float)v;
      }
    }
    return;
  }
  // R[a][c] = U[a][c] / sqrt(d_a) for c >= a (coalesced: consecutive threads, consecutive c).
  // R^-1[c][a] = E[a][c] / sqrt(d_a) for c <= a: transposed through LDS.
#pragma unroll
  for (int ia = 0; ia < 4; ++ia) {
    const int a = tr + 32 * ia;
    if (a >= l) continue;
    const double rs = 1.0 / sqrt(diag[a]);
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) {
      const int c = tc + 32 * ib;
      if (c >= l) continue;
      if (p.R) p.R[(int64_t)a * l + c] = c >= a ? U[ia][ib] * rs : 0.0;
      tbuf[c * TLD + a] = c == a ? rs : (c < a ? E[ia][ib] * rs : 0.0);
    }
  }
  __syncthreads();
  for (int idx = tid; idx < l * l; idx += 1024) {
    const int row = idx / l, col = idx - row * l;
    const double v = tbuf[row * TLD + col];
    if (p.Rinv) p.Rinv[idx] = v;
    if (p.RinvT) {
      if (p.dtype == RSVD_F64) ((double*)p.RinvT)[idx] = v;
      else ((float*)p.RinvT)[idx] = (float)v;
    }
  }
}

__global__ __launch_bounds__(1024) void chol_kernel(const CholParams p) { chol_body(p, blockIdx.x); }

__global__ __launch_bounds__(1024) void chol_batched(const CholParams* __restrict__ ps, const BlockMap* __restrict__ bm) {
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
  hipLaunchKernelGGL(chol_batched, dim3((unsigned)nblocks), dim3(1024), 0, st, ps, bm);
  return hipGetLastError();
}

hipError_t launch_chol(const CholParams& p, hipStream_t st) {
  if (p.l > 128 || p.l < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(1024), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_trmm_upper(const double* R2, const double* R1, double* R, int32_t l, const int32_t* gate,
                             hipStream_t st) {
  const TrmmParams p{R2, R1, R, l, gate};
  hipLaunchKernelGGL(trmm_upper_kernel, dim3((unsigned)trmm_blocks(p)), dim3(256), 0, st, p);
  return hipGetLastError();
}

}  // namespace rsvd
