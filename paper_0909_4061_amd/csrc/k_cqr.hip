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
// threads.  With L = R^T, the row operations that take W to R (block row k
// scaled by L_kk^-1, then subtracted from the rows below it) take I to L^-1 =
// X^T, so both come out of the same passes.  One LDS matrix holds both parts:
// the upper triangle holds W, then R; the strict lower triangle holds the
// eliminated identity, then X^T; its diagonal (1 / R_ii) is kept in a vector.
//
// Per block of CB rows [k0, k1):
//   1. panel, one wave: the diagonal block is factored in registers
//      (right-looking, pivots and rows of R_kk broadcast within each 16-lane
//      row by DPP; every row of lanes holds a copy), and every other column of
//      the block row -- R part right of the block, identity part left of and
//      inside it -- is multiplied by R_kk^-T, two columns per lane.  The
//      finished block row is also staged in a separate LDS buffer;
//   2. trailing update of rows k1..l-1 from the staged block row, both parts at
//      once (columns below k1: identity part; columns >= the row: R part), in
//      4 x 4 register tiles fed by 16-byte LDS reads.
// A pivot that is not positive (or not finite) restarts the factorization on
// W + s I with the shifted-CholeskyQR shift; a second failure (non-finite
// input) returns identity factors and raises RSVD_FLAG_NONFINITE.

// 1/sqrt(x) from the hardware estimate and two Newton steps (x > 0, finite).
__device__ __forceinline__ double rsq_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

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

template <int CB>
__device__ __forceinline__ void chol_body_t(const CholParams& p) {
  static_assert(CB == 16, "the trailing update tiles are 16 x 16");
  constexpr int NT = 512, NW = NT / 64, LDC = 130;  // even: rows start on 16-byte boundaries
  constexpr int PLD = 144;                          // staged row: 128 columns + tile overhang
  __shared__ __attribute__((aligned(16))) double M[128 * LDC];
  __shared__ __attribute__((aligned(16))) double Pr[CB * PLD];
  __shared__ double rinv_d[128];  // 1 / R_ii (0 past l)
  __shared__ int bad_s;
  if (p.gate && *p.gate == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0 && p.shifted && p.reset_shifted) *p.shifted = 0;  // set again below by the same thread
  const int l = p.l, Lg = p.Lg;
  const int lp = (l + 15) & ~15;            // rows and columns past l up to lp hold zeros
  const int tc = tid & 127, tr = tid >> 7;  // 4 x 128 thread grid for whole-matrix loops
  const double eps = DBL_EPSILON;

  double thresh = 0.0, trace = 0.0;
  bool ok = false;
  for (int attempt = 0; attempt < 2 && !ok; ++attempt) {
    // Shifted CholeskyQR: s = 11 (rows l + l (l + 1)) u ||Y||_F^2 with u the FP64 unit roundoff.
    const double shift =
        attempt == 0 ? 0.0 : 11.0 * ((double)p.rows * l + (double)l * (l + 1)) * (0.5 * eps) * trace;
    {
      // column pair 2 (tid % 64), rows tid / 64 + 8 u: every load in flight at once
      const int cp = 2 * (tid & 63), r0 = tid >> 6;
      dbl2 v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int a = r0 + 8 * u;
        v[u] = (a < l && cp + 1 >= a && cp < l) ? *reinterpret_cast<const dbl2*>(p.G + (int64_t)a * Lg + cp)
                                                : dbl2{0.0, 0.0};
      }
      if (attempt == 0) {
        // max diagonal (breakdown threshold) and trace (shift) of W, every wave for
        // itself, while the loads above are in flight
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
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int a = r0 + 8 * u;
        if (a < lp && cp < lp) {
          dbl2 w = v[u];
          w.x = (cp < l && cp >= a) ? w.x + (cp == a ? shift : 0.0) : 0.0;
          w.y = (cp + 1 < l && cp + 1 >= a) ? w.y + (cp + 1 == a ? shift : 0.0) : 0.0;
          *reinterpret_cast<dbl2*>(M + a * LDC + cp) = w;
        }
      }
    }
    for (int i = tid; i < CB * PLD; i += NT) Pr[i] = 0.0;
    if (tid < 128) rinv_d[tid] = 0.0;
    __syncthreads();
    ok = true;
    for (int k0 = 0; k0 < l; k0 += CB) {
      const int k1 = min(k0 + CB, l), bk = k1 - k0;
      // 1. panel by waves 0 and 1.  Both factor the diagonal block (each 16-lane row
      //    of both waves holds a copy); column sc = lane + 64 wave of the block row
      //    is multiplied by R_kk^-T in the lane's registers.  Every load and store
      //    stays inside M and Pr: values read from the zero padding or past lp only
      //    ever reach entries that no later step reads.
      const int dq = lane & (CB - 1);  // diagonal column k0 + dq
      const int sc = lane + 64 * wave;
      const bool diag = sc >= k0 && sc < k1;  // identity column inside the block: then dq == sc - k0
      double x0[CB], xt[CB];
      if (wave < 2) {
#pragma unroll
        for (int i = 0; i < CB; ++i) {
          x0[i] = M[(k0 + i) * LDC + k0 + dq];  // below the diagonal: never read by other lanes
          const double w = M[(k0 + i) * LDC + sc];
          xt[i] = diag ? (i == dq ? 1.0 : 0.0) : w;
        }
      }
      __syncthreads();  // both waves hold the diagonal block before either stores into it
      if (wave < 2) {
        double rv = 0.0;
        bool bad = false;
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          if (j < bk) {  // uniform; a failed pivot only sets bad (the results are discarded)
            const double djj = row_bcast_at(x0[j], j);
            bad = bad || !(djj > thresh) || !isfinite(djj);
            const double rinv = rsq_refined(djj);
            double rjj = djj * rinv;
            rjj = fma(0.5 * rinv, fma(-rjj, rjj, djj), rjj);
            x0[j] = dq == j ? rjj : x0[j] * rinv;  // row j of R_kk
            rv = dq == j ? rinv : rv;
            xt[j] *= rinv;
#pragma unroll
            for (int i = j + 1; i < CB; ++i) {
              const double rji = row_bcast_at(x0[j], i);  // R[j][i]
              x0[i] = fma(-rji, x0[j], x0[i]);
              xt[i] = fma(-rji, xt[j], xt[i]);
            }
          }
        }
        if (!bad) {
          // identity columns inside the block carry R_kk above the diagonal (the
          // lane's copy of column k0 + dq) and X_kk^T below it
#pragma unroll
          for (int i = 0; i < CB; ++i) {
            M[(k0 + i) * LDC + sc] = (diag && i <= dq) ? x0[i] : xt[i];
            Pr[i * PLD + sc] = xt[i];
          }
          if (diag) rinv_d[sc] = rv;
        }
        if (tid == 0) bad_s = bad ? 1 : 0;
      }
      __syncthreads();
      if (bad_s) {
        ok = false;
        break;
      }
      // 2. trailing update, one 16 x 16 output tile per wave and step, on FP64 MFMA
      //    (K = 16: four 16x16x4 products).  Row tile r (rows k1 + 16 r ..) needs
      //    the identity-part tiles left of k1 and the R-part tiles from its own
      //    diagonal tile on: lp/16 - r tiles.
      if (k1 < l) {
        const int T = lp / 16, K1 = k1 / 16, nrt = T - K1;
        const int items = nrt * T - nrt * (nrt - 1) / 2;
        for (int it = wave; it < items; it += NW) {
          int r = 0, u = it;
          while (u >= T - r) {  // uniform: at most 8 steps
            u -= T - r;
            ++r;
          }
          const int cj = u < K1 ? u : u + r;
          const int ib = k1 + 16 * r, cb = 16 * cj;
          const int li = lane & 15, lk = lane >> 4;
          f64x4 acc = f64x4{};
#pragma unroll
          for (int s4 = 0; s4 < CB / 4; ++s4) {
            const double* row = Pr + (4 * s4 + lk) * PLD;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(row[ib + li], row[cb + li], acc, 0, 0, 0);
          }
          // acc[e] belongs to row ib + 4 e + lk, column cb + li
          const int c = cb + li;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int i = ib + 4 * e + lk;
            if (i < l && c < l && (c < k1 || c >= i)) M[i * LDC + c] -= acc[e];
          }
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
  if (tc < l)
    for (int a = tr; a < l; a += 4) {
      const int64_t idx = (int64_t)a * l + tc;
      if (p.R) p.R[idx] = tc >= a ? M[a * LDC + tc] : 0.0;
      // X[a][tc] = (X^T)[tc][a]
      const double v = tc > a ? M[tc * LDC + a] : (tc == a ? rinv_d[a] : 0.0);
      if (p.Rinv) p.Rinv[idx] = v;
      if (p.RinvT) {
        if (p.dtype == RSVD_F64) ((double*)p.RinvT)[idx] = v;
        else ((float*)p.RinvT)[idx] = (float)v;
      }
    }
}

__device__ __forceinline__ void chol_body(const CholParams& p, const int bid) {
  (void)bid;  // one workgroup per factorization
  chol_body_t<16>(p);
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
