// CholeskyQR building blocks: the orthonormalization "Y = QR" that follows
// every application of A or A* in Stage A (Algorithm 4.1 step 3, Algorithm 4.4
// steps 2, 4, 5; Section 4.1 allows any stable QR).  One CholeskyQR pass is
//   W = Y^T Y (FP64),  W = R^T R (Cholesky),  Q = Y R^-1,
// and CholeskyQR2 repeats it once on Q.  The host chains these kernels:
//
//   sum_parts    : sums the split-K partial products of the GEMM that made Y
//                  (fixed order) and stores Y.
//   gram_partial : one workgroup per (row chunk, group of upper 16x16 tiles):
//                  the chunk's rows are staged 64 at a time through LDS and
//                  the block Gram Y_c^T Y_c accumulated on FP64 MFMA (FP32
//                  entries are exact in FP64, so the products are exact).
//                  A single Gram splits its tiles over several workgroups
//                  per chunk so that it fills the chip with few partials; a
//                  batch of Grams uses 64-row chunks with every tile.
//   gram_reduce  : sums the chunk Grams in a fixed order (deterministic).
//   chol         : one workgroup of 512 threads.  R and R^-1 together by
//                  blocked (by 16) elimination on [W | I] in LDS: a panel in
//                  registers, trailing tiles on FP64 MFMA, two barriers per
//                  block.
//                  A pivot that is not safely positive restarts the
//                  factorization on W + sI (shifted CholeskyQR) and raises a
//                  flag; the host then runs a third pass.
//   trmm_upper   : R = R2 R1 for the combined factor.
#include <float.h>

#include "common.hpp"

namespace rsvd {

namespace {

// Split-K partial sums: one thread per 16 bytes of a row, every partial's load
// in flight at once, summed in the order s = 0, 1, ... (deterministic).
template <typename T>
__device__ __forceinline__ void sum_parts_body(const GramParams& p, const int bid) {
  constexpr int V = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(V)));
  if (p.gate && *p.gate == 0) return;
  const int per_row = (p.l + V - 1) / V;
  const int64_t idx = (int64_t)bid * 256 + threadIdx.x;
  const int64_t row = idx / per_row;
  const int cv = (int)(idx - row * per_row) * V;
  if (row >= p.rows) return;
  const T* __restrict__ part = (const T*)p.part;
  vec v[16];
#pragma unroll
  for (int s = 0; s < 16; ++s)
    if (s < p.S) v[s] = *reinterpret_cast<const vec*>(part + ((int64_t)s * p.rows + row) * p.Lp + cv);
  vec acc = v[0];
#pragma unroll
  for (int s = 1; s < 16; ++s)
    if (s < p.S) acc += v[s];
  T* __restrict__ y = (T*)p.yout;
#pragma unroll
  for (int e = 0; e < V; ++e)
    if (cv + e < p.l) y[row * p.ldy + cv + e] = acc[e];
}

template <typename T>
__global__ __launch_bounds__(256) void sum_parts_kernel(const GramParams p) { sum_parts_body<T>(p, blockIdx.x); }

template <typename T>
__global__ __launch_bounds__(256) void sum_parts_batched(const GramParams* __restrict__ ps,
                                                         const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  sum_parts_body<T>(ps[b.item], b.local);
}

// Partial Gram of one row chunk for one group of 16 x 16 tiles (upper
// triangle, tiles t = group, group + tgroups, ...; wave w of the workgroup
// takes every fourth of them), accumulated over the chunk's 64-row stages on
// FP64 MFMA.  FP32 entries are exact in FP64, so the products are exact.  The
// next stage's rows are loaded into registers while the current one is
// multiplied.
template <typename T>
__device__ __forceinline__ void gram_partial_body(const GramParams& p, const int bid) {
  constexpr int RB = GRAM_ROWS;
  // Row stride of the staged rows: 144 = 16 modulo the 64 banks, so the four
  // rows of 16 consecutive elements that one MFMA operand read takes fall on
  // four disjoint quarters of the banks (129 put them one bank apart: four
  // lanes per bank).
  constexpr int YLD = 144;
  constexpr int MAXT = 9;  // tiles per wave: 36 tiles / 4 waves with one group
  __shared__ T Ys[RB * YLD];
  if (p.gate && *p.gate == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l = p.l, Lg = p.Lg, G = p.tgroups;
  const int chunk = bid / G, grp = bid - chunk * G;
  const int64_t rbeg = (int64_t)chunk * p.chunk;
  const int64_t rend = min(p.rows, rbeg + p.chunk);
  const int nt = Lg / 16, ntiles = nt * (nt + 1) / 2;

  // this wave's tiles: v_mfma_f64_16x16x4f64 with A[i = lane%16][k = lane/16] =
  // Y[k][16 ti + i], B[k = lane/16][j = lane%16] = Y[k][16 tj + j]; result register
  // e of lane holds G[16 ti + 4 e + lane/16][16 tj + lane%16]
  int ti[MAXT], tj[MAXT];
#pragma unroll
  for (int j = 0; j < MAXT; ++j) {
    int rem = grp + G * (wave + 4 * j), r = 0;
    if (rem >= ntiles) rem = 0;
    while (rem >= nt - r) {
      rem -= nt - r;
      ++r;
    }
    ti[j] = r;
    tj[j] = r + rem;
  }
  f64x4 acc[MAXT];
#pragma unroll
  for (int j = 0; j < MAXT; ++j) acc[j] = f64x4{};

  // stage loads: column tid % 128 of rows tid / 128 + 2 it
  constexpr int ITER = RB * 128 / 256;
  const int c = tid & 127, rb = tid >> 7;
  const T* __restrict__ yin = (const T*)p.yin;
  T vals[ITER];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int64_t row = rbeg + rb + 2 * it;
    vals[it] = (row < rend && c < l) ? yin[row * p.ldy + c] : (T)0;
  }
  for (int64_t r0 = rbeg; r0 < rend; r0 += RB) {
    __syncthreads();  // the previous stage's products are done with Ys
    if (c < Lg) {
#pragma unroll
      for (int it = 0; it < ITER; ++it) Ys[(rb + 2 * it) * YLD + c] = vals[it];
    }
    __syncthreads();
    if (r0 + RB < rend) {
#pragma unroll
      for (int it = 0; it < ITER; ++it) {
        const int64_t row = r0 + RB + rb + 2 * it;
        vals[it] = (row < rend && c < l) ? yin[row * p.ldy + c] : (T)0;
      }
    }
#pragma unroll
    for (int j = 0; j < MAXT; ++j) {
      if (grp + G * (wave + 4 * j) < ntiles) {  // uniform across the wave
#pragma unroll 4
        for (int ks = 0; ks < RB / 4; ++ks) {
          const int kr = 4 * ks + (lane >> 4);
          const double a = (double)Ys[kr * YLD + 16 * ti[j] + (lane & 15)];
          const double b = (double)Ys[kr * YLD + 16 * tj[j] + (lane & 15)];
          acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
        }
      }
    }
  }
  double* gout = p.gpart + (int64_t)chunk * Lg * Lg;
#pragma unroll
  for (int j = 0; j < MAXT; ++j) {
    if (grp + G * (wave + 4 * j) < ntiles) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        gout[(int64_t)(16 * ti[j] + 4 * e + (lane >> 4)) * Lg + 16 * tj[j] + (lane & 15)] = acc[j][e];
    }
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
  if (live) {
#pragma unroll 8
    for (int64_t b = q; b < p.nblk; b += 4) acc += p.gpart[b * LL + e];
  }
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
// inverse X = R^-1, by blocked elimination on [W | I] for one workgroup of 512
// threads (8 waves).  With L = R^T, the row operations that take W to R (block
// row k scaled by L_kk^-1, then subtracted from the rows below it) take I to
// L^-1 = X^T, so both come out of the same passes.  One LDS matrix holds both
// parts: the upper triangle holds W, then R; the strict lower triangle holds the
// eliminated identity, then X^T; its diagonal (1 / R_ii) is kept in a vector.
//
// Blocks of 16 rows, with one block of look-ahead.  Iteration k:
//   1. (k > 0) the rows of block k receive the update from block k - 1, one
//      16 x 16 tile per wave on FP64 MFMA;
//   2. waves 0 and 1 factor block k (the panel: its diagonal block in registers,
//      pivots and rows of R_kk broadcast within each 16-lane row by DPP, every
//      other column of the block row multiplied by R_kk^-T in the same steps, one
//      column per lane) and write its rows of R and columns of R^-1 to global
//      memory, while waves 2..7 apply the update from block k - 1 to the rows
//      below block k, two tiles at a time.
// So the serial chain of the factorization (the panels) overlaps the trailing
// updates; block 0 is read from global memory by the panel waves while the
// other waves load the rest of W.  A pivot that is not positive (or not finite)
// restarts the factorization on W + s I with the shifted-CholeskyQR shift; a
// second failure (non-finite input) returns identity factors and raises
// RSVD_FLAG_NONFINITE.

// Value of lane L of this lane's 16-lane row (DPP row_newbcast).
template <int L>
__device__ __forceinline__ double row_bcast(double v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + L, 0xF, 0xF, false);
}

// Lane index as an ordinary argument: call it only with values the unrolled
// loops make constant, so that the switch folds to one DPP move.
__device__ __forceinline__ double row_bcast_at(double v, int L) {
  switch (L) {
    case 0: return row_bcast<0>(v);
    case 1: return row_bcast<1>(v);
    case 2: return row_bcast<2>(v);
    case 3: return row_bcast<3>(v);
    case 4: return row_bcast<4>(v);
    case 5: return row_bcast<5>(v);
    case 6: return row_bcast<6>(v);
    case 7: return row_bcast<7>(v);
    case 8: return row_bcast<8>(v);
    case 9: return row_bcast<9>(v);
    case 10: return row_bcast<10>(v);
    case 11: return row_bcast<11>(v);
    case 12: return row_bcast<12>(v);
    case 13: return row_bcast<13>(v);
    case 14: return row_bcast<14>(v);
    default: return row_bcast<15>(v);
  }
}

typedef double dbl2 __attribute__((ext_vector_type(2)));

// 1/sqrt(d) from the hardware estimate y0 (relative error e ~ 2^-24) by one step of
// the third-order series d^-1/2 = y0 (1 - e)^-1/2 = y0 (1 + e/2 + 3e^2/8 + O(e^3)),
// e = 1 - d y0^2: error O(e^3) below the FP64 rounding, four dependent operations.
__device__ __forceinline__ double rsq_series(double d) {
  const double y0 = __builtin_amdgcn_rsq(d);
  const double e = fma(-(d * y0), y0, 1.0);
  return fma(y0 * e, fma(0.375, e, 0.5), y0);
}

constexpr int CHOL_LDC = 130;
constexpr int CHOL_UPDATE_WAVES = 6;

// Panel factorization of rows [k0, k0 + 16) for waves 0 and 1: column sc = lane + 64 wave of the
// block row in xt[], a copy of column dq = lane % 16 of the diagonal block in x0[] (every 16-lane
// row holds one; entries below a lane's diagonal are never read).  Straight-line code: a padded
// pivot (row >= l) holds 1 and changes nothing.  Writes the rows to M, 1/R_jj to rinv_d, and the
// finished rows of R and columns of R^-1 to global memory.  Returns true when a pivot failed.
__device__ __forceinline__ bool chol_panel(const CholParams& p, double* M, double* rinv_d, const int k0, const int l,
                                          const double thresh, double (&x0)[16], double (&xt)[16]) {
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));  // keep the lane masks below inside the panel loop
  const int wave = threadIdx.x >> 6;
  const int dq = lane & 15, sc = lane + 64 * wave;
  const int bk = min(16, l - k0);
  const bool diag = sc >= k0 && sc < k0 + 16;
  double rv = 0.0, rd = 0.0, pmin = DBL_MAX;
  bool nonfinite = false;
  // Software-pipelined: the next pivot is broadcast and its reciprocal square root started as
  // soon as it has its last update.  The asm statements pin every update of a step inside that
  // step (no sinking into the next one, which would keep every broadcast live across steps).
  double y = rsq_series(row_bcast_at(x0[0], 0));
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const double d = row_bcast_at(x0[j], j);
    if (j < bk) {
      pmin = d < pmin ? d : pmin;
      nonfinite |= !isfinite(d);
    }
    x0[j] *= y;
    xt[j] *= y;
    double ynext = 1.0;
    if (j + 1 < 16) {
      const double r = row_bcast_at(x0[j], j + 1);
      x0[j + 1] = fma(-r, x0[j], x0[j + 1]);
      xt[j + 1] = fma(-r, xt[j], xt[j + 1]);
      ynext = rsq_series(row_bcast_at(x0[j + 1], j + 1));
    }
#pragma unroll
    for (int i = j + 2; i < 16; ++i) {
      const double r = row_bcast_at(x0[j], i);
      x0[i] = fma(-r, x0[j], x0[i]);
      xt[i] = fma(-r, xt[j], xt[i]);
    }
    double rjj = d * y;
    rjj = fma(0.5 * y, fma(-rjj, rjj, d), rjj);
    rd = dq == j ? rjj : rd;
    rv = dq == j ? y : rv;
    y = ynext;
#pragma unroll
    for (int i = j; i < 16; ++i) asm volatile("" : "+v"(x0[i]), "+v"(xt[i]));
    asm volatile("" : "+v"(rd), "+v"(rv), "+v"(pmin));
    __builtin_amdgcn_sched_barrier(0);
  }
  const bool bad = !(pmin > thresh) || nonfinite;
  if (!bad) {
#pragma unroll
    for (int i = 0; i < 16; ++i) M[(k0 + i) * CHOL_LDC + sc] = xt[i];
    if (diag) {
      // the diagonal block: R_kk on and above the diagonal, R_kk^-T below it
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (i <= dq) M[(k0 + i) * CHOL_LDC + sc] = i == dq ? rd : x0[i];
      rinv_d[sc] = rv;
    }
    if (sc < l) {
      // row block of R: R[k0 + i][sc] (coalesced across lanes); zero left of the block
      if (p.R) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (i < bk)
            p.R[(int64_t)(k0 + i) * l + sc] =
                sc < k0 ? 0.0 : (diag ? (i < dq ? x0[i] : (i == dq ? rd : 0.0)) : xt[i]);
      }
      // column block of X = R^-1: X[sc][k0 + i], i < bk: 16 consecutive entries per lane (zero
      // right of the block; R_kk^-T is exactly zero above its diagonal), with 16-byte stores
      // when the row offsets allow it
      const bool zero = sc >= k0 + 16;
      const int64_t xo = (int64_t)sc * l + k0;
      if (p.RinvT && p.dtype != RSVD_F64) {
        float* dst = (float*)p.RinvT + xo;
        if ((l & 3) == 0 && (reinterpret_cast<uintptr_t>(p.RinvT) & 15) == 0) {
          if (zero) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (4 * q < bk) *reinterpret_cast<float4*>(dst + 4 * q) = make_float4(0.f, 0.f, 0.f, 0.f);
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (4 * q < bk)
                *reinterpret_cast<float4*>(dst + 4 * q) =
                    make_float4((float)xt[4 * q], (float)xt[4 * q + 1], (float)xt[4 * q + 2], (float)xt[4 * q + 3]);
          }
        } else {
#pragma unroll
          for (int i = 0; i < 16; ++i)
            if (i < bk) dst[i] = zero ? 0.f : (float)xt[i];
        }
      }
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        double* base = w == 0 ? p.Rinv : (p.dtype == RSVD_F64 ? (double*)p.RinvT : nullptr);
        if (!base) continue;
        double* dst = base + xo;
        if ((l & 1) == 0 && (reinterpret_cast<uintptr_t>(base) & 15) == 0) {
          if (zero) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
              if (2 * q < bk) *reinterpret_cast<dbl2*>(dst + 2 * q) = dbl2{0.0, 0.0};
          } else {
#pragma unroll
            for (int q = 0; q < 8; ++q)
              if (2 * q < bk) *reinterpret_cast<dbl2*>(dst + 2 * q) = dbl2{xt[2 * q], xt[2 * q + 1]};
          }
        } else {
#pragma unroll
          for (int i = 0; i < 16; ++i)
            if (i < bk) dst[i] = zero ? 0.0 : xt[i];
        }
      }
    }
  }
  return bad;
}

// NTL 16 x 16 output tiles (row tile t[q], column tile cj[q]; a tile with t[q] < 0 is skipped)
// of the trailing update from panel k: M[i][c] -= sum_s X[s][i] X[s][c], X = rows [k0, k0 + 16)
// of M (the identity columns of the panel itself read R_kk^-T: strictly lower part from M,
// diagonal from rinv_d, zero above).  Every operand of every tile is read before the first
// product, two accumulators per tile.
template <int NTL>
__device__ __forceinline__ void chol_tiles(double* M, const double* rinv_d, const int k, const int (&t)[NTL],
                                          const int (&cj)[NTL], const int l) {
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
  const int li = lane & 15, lk = lane >> 4;
  const int k0 = 16 * k, k1 = k0 + 16;
  double a[NTL][4], b[NTL][4], mo[NTL][4], rvv[4];
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) rvv[s4] = rinv_d[k0 + 4 * s4 + lk];
#pragma unroll
  for (int q = 0; q < NTL; ++q) {
    const int tq = t[q] < 0 ? k + 1 : t[q];  // a skipped tile reads valid rows
    const int ib = 16 * tq, c = 16 * cj[q] + li;
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const double* row = M + (k0 + 4 * s4 + lk) * CHOL_LDC;
      a[q][s4] = row[ib + li];
      b[q][s4] = row[c];
      mo[q][s4] = M[(ib + 4 * s4 + lk) * CHOL_LDC + c];
    }
  }
#pragma unroll
  for (int q = 0; q < NTL; ++q)
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) asm volatile("" : "+v"(a[q][s4]), "+v"(b[q][s4]), "+v"(mo[q][s4]));
  f64x4 acc[NTL][2];
#pragma unroll
  for (int q = 0; q < NTL; ++q) acc[q][0] = acc[q][1] = f64x4{};
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
    for (int q = 0; q < NTL; ++q) {
      const int s = 4 * s4 + lk;
      const double bb = cj[q] == k ? (li < s ? b[q][s4] : (li == s ? rvv[s4] : 0.0)) : b[q][s4];
      acc[q][s4 & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q][s4], bb, acc[q][s4 & 1], 0, 0, 0);
    }
#pragma unroll
  for (int q = 0; q < NTL; ++q) {
    if (t[q] < 0) continue;
    const f64x4 s = acc[q][0] + acc[q][1];
    const int ib = 16 * t[q], c = 16 * cj[q] + li;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = ib + 4 * e + lk;
      if (i < l && c < l && (c < k1 || c >= i)) M[i * CHOL_LDC + c] = mo[q][e] - s[e];
    }
  }
}

__device__ __forceinline__ void chol_body(const CholParams& p, const int bid) {
  (void)bid;  // one workgroup per factorization
  constexpr int LDC = CHOL_LDC;
  __shared__ __attribute__((aligned(16))) double M[128 * LDC];
  __shared__ double rinv_d[128];
  __shared__ int bad_s;
  if (p.gate && *p.gate == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0 && p.shifted && p.reset_shifted) *p.shifted = 0;
  const int l = p.l, Lg = p.Lg;
  const int lp = (l + 15) & ~15, T = lp >> 4;
  const int tc = tid & 127, tr = tid >> 7;
  const double eps = DBL_EPSILON;
  // breakdown threshold (panel waves) and shift (all waves, only after a failure) from the
  // diagonal of W
  auto diag_stats = [&](double& mx_out, double& tr_out) {
    const double d0 = lane < l ? p.G[(int64_t)lane * (Lg + 1)] : 0.0;
    const double d1 = lane + 64 < l ? p.G[(int64_t)(lane + 64) * (Lg + 1)] : 0.0;
    double mx = fmax(d0, d1), trs = d0 + d1;
    for (int off = 32; off > 0; off >>= 1) {
      mx = fmax(mx, __shfl_xor(mx, off, 64));
      trs += __shfl_xor(trs, off, 64);
    }
    mx_out = mx;
    tr_out = trs;
  };
  double thresh = 0.0, trace = 0.0;
  bool ok = false;
  for (int attempt = 0; attempt < 2 && !ok; ++attempt) {
    if (attempt == 1 && wave >= 2) {
      double mx;
      diag_stats(mx, trace);
    }
    const double shift =
        attempt == 0 ? 0.0 : 11.0 * ((double)p.rows * l + (double)l * (l + 1)) * (0.5 * eps) * trace;
    ok = true;
    for (int k = 0; ok && 16 * k < l; ++k) {
      if (k > 0) {
        // rows of this panel first, one tile per wave, from the panel before
        if (wave < T) {
          const int tt[1] = {k}, cc[1] = {wave};
          chol_tiles<1>(M, rinv_d, k - 1, tt, cc, l);
        }
        __syncthreads();
      }
      int ln = lane;
      asm volatile("" : "+v"(ln));  // addresses below are formed here, not hoisted and spilled
      if (wave < 2) {
        const int dq = ln & 15, sc = ln + 64 * wave, k0 = 16 * k;
        double x0[16], xt[16];
        if (k == 0) {
          // the first panel straight from W in global memory, while waves 2.. load the rest
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            x0[i] = (i <= dq && dq < l) ? p.G[(int64_t)i * Lg + dq] : 0.0;
            xt[i] = (i < l && sc >= 16 && sc < l) ? p.G[(int64_t)i * Lg + sc] : 0.0;
          }
          if (attempt == 0) {
            double mx;
            diag_stats(mx, trace);
            thresh = (double)l * 16.0 * eps * mx;
          }
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            asm volatile("" : "+v"(x0[i]), "+v"(xt[i]));
            x0[i] = i != dq ? x0[i] : (dq < l ? x0[i] + shift : 1.0);
            xt[i] = sc < 16 ? (i == dq ? 1.0 : 0.0) : xt[i];
          }
        } else {
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            x0[i] = M[(k0 + i) * LDC + k0 + dq];
            xt[i] = M[(k0 + i) * LDC + sc];
          }
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            asm volatile("" : "+v"(xt[i]));
            xt[i] = (sc >= k0 && sc < k0 + 16) ? (i == dq ? 1.0 : 0.0) : xt[i];
          }
        }
        const bool bad = chol_panel(p, M, rinv_d, k0, l, thresh, x0, xt);
        if (tid == 0) bad_s = bad ? 1 : 0;
      } else if (k == 0) {
        // rows 16.. of W (upper triangle, shifted diagonal; zeros below; padded rows hold 1 on
        // the diagonal) into M, two columns per thread
        const int cp = 2 * ln, r0 = 16 + (wave - 2);
        dbl2 v[19];
#pragma unroll
        for (int u = 0; u < 19; ++u) {
          const int a = r0 + 6 * u;
          v[u] = (a < l && cp + 1 >= a && cp < l) ? *reinterpret_cast<const dbl2*>(p.G + (int64_t)a * Lg + cp)
                                                  : dbl2{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < 19; ++u) {
          const int a = r0 + 6 * u;
          if (a < 128) {
            dbl2 w = v[u];
            w.x = (cp < l && cp >= a) ? w.x + (cp == a ? shift : 0.0) : (cp == a ? 1.0 : 0.0);
            w.y = (cp + 1 < l && cp + 1 >= a) ? w.y + (cp + 1 == a ? shift : 0.0) : (cp + 1 == a ? 1.0 : 0.0);
            *reinterpret_cast<dbl2*>(M + a * LDC + cp) = w;
          }
        }
      } else {
        // the rest of the update from panel k - 1: row tiles t >= k + 1 (k identity tiles and
        // T - t R tiles each), items wave - 2, wave + 4, ... of that list, two at a time
        int t = k + 1, u = wave - 2;
        while (t < T) {
          int tt[2], cc[2];
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            int cnt = k + (T - t);
            while (t < T && u >= cnt) {
              u -= cnt;
              ++t;
              cnt = k + (T - t);
            }
            tt[q] = t < T ? t : -1;
            cc[q] = t < T ? (u < k ? u : t + (u - k)) : 0;
            u += CHOL_UPDATE_WAVES;
          }
          if (tt[0] >= 0) chol_tiles<2>(M, rinv_d, k - 1, tt, cc, l);
        }
      }
      __syncthreads();
      ok = bad_s == 0;
    }
    if (!ok && attempt == 0 && tid == 0) {
      atomicOr(p.status, (int32_t)RSVD_FLAG_SHIFTED);
      if (p.shifted) *p.shifted = 1;
    }
    __syncthreads();
  }
  if (!ok) {
    if (tid == 0) atomicOr(p.status, (int32_t)RSVD_FLAG_NONFINITE);
    if (tc < l)
      for (int a = tr; a < l; a += 4) {
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

int64_t gram_geometry(int64_t rows, int32_t Lg, bool wide, int32_t* tgroups, int32_t* chunk) {
  const int nt = Lg / 16, ntiles = nt * (nt + 1) / 2;
  const int64_t nsub = (rows + GRAM_ROWS - 1) / GRAM_ROWS;
  if (!wide) {
    *tgroups = 1;
    *chunk = (int32_t)((nsub < 2 ? nsub : 2) * GRAM_ROWS);
    return (rows + *chunk - 1) / *chunk;
  }
  const int G = ntiles > 12 ? (ntiles + 11) / 12 : 1;  // at most three tiles per wave
  const int64_t want = (256 + G - 1) / G;                // chunks that fill 256 CUs
  const int64_t nch = nsub < want ? nsub : want;
  const int64_t per = nch > 0 ? (nsub + nch - 1) / nch : 1;
  *tgroups = G;
  *chunk = (int32_t)(per * GRAM_ROWS);
  return (rows + *chunk - 1) / *chunk;
}

namespace {
bool gram_params_ok(const GramParams& p) {
  const int nt = p.Lg / 16;
  return p.l <= 128 && p.Lg % 16 == 0 && p.Lg >= p.l && p.tgroups >= 1 && p.chunk >= GRAM_ROWS &&
         p.chunk % GRAM_ROWS == 0 && nt * (nt + 1) / 2 <= 36 * p.tgroups;
}
}  // namespace

hipError_t launch_gram_partial(int dtype, const GramParams& p, hipStream_t st) {
  if (p.rows <= 0) return hipSuccess;
  if (!gram_params_ok(p)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)gram_partial_blocks(p));
  if (dtype == RSVD_F64)
    hipLaunchKernelGGL(gram_partial_kernel<double>, grid, dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(gram_partial_kernel<float>, grid, dim3(256), 0, st, p);
  return hipGetLastError();
}

bool sum_parts_ok(int dtype, const GramParams& p) {
  const int V = dtype == RSVD_F64 ? 2 : 4;
  return p.S >= 1 && p.S <= 16 && p.Lp % V == 0 && p.Lp >= p.l && p.l >= 1;
}

int64_t sum_parts_blocks(int dtype, const GramParams& p) {
  const int V = dtype == RSVD_F64 ? 2 : 4;
  return p.rows <= 0 ? 0 : (p.rows * ((p.l + V - 1) / V) + 255) / 256;
}

hipError_t launch_sum_parts(int dtype, const GramParams& p, hipStream_t st) {
  if (p.rows <= 0) return hipSuccess;
  if (!sum_parts_ok(dtype, p)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)sum_parts_blocks(dtype, p));
  if (dtype == RSVD_F64)
    hipLaunchKernelGGL(sum_parts_kernel<double>, grid, dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(sum_parts_kernel<float>, grid, dim3(256), 0, st, p);
  return hipGetLastError();
}

int64_t gram_partial_blocks(const GramParams& p) { return (p.rows + p.chunk - 1) / p.chunk * p.tgroups; }

int64_t gram_reduce_blocks(const GramReduceParams& p) { return ((int64_t)p.Lg * p.Lg + 63) / 64; }

hipError_t launch_gram_reduce(const double* gpart, int64_t nblk, int32_t Lg, double* G, int32_t* status,
                              const int32_t* gate, hipStream_t st) {
  const GramReduceParams p{gpart, nblk, Lg, G, status, gate};
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)gram_reduce_blocks(p)), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_sum_parts_batched(int dtype, const GramParams* ps, const BlockMap* bm, int64_t nblocks,
                                    hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (dtype == RSVD_F64)
    hipLaunchKernelGGL(sum_parts_batched<double>, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
  else
    hipLaunchKernelGGL(sum_parts_batched<float>, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
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
