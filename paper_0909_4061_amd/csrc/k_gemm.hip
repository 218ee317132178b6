// Tall-skinny GEMMs that stream A: the sketch Y = A Omega (Algorithm 4.1,
// step 2), the power steps A* Q and A Qt (Algorithm 4.4, steps 4-5), the
// projection B = Q* A (Algorithm 5.1, step 1, written as Bt = A^T Q), and the
// small right-hand products of CholeskyQR (Y R^-1) and of the lifts (Q U~).
//
// Every variant computes C (rows x ncols, ncols <= 128) = op(A) X with one
// workgroup per block of `bm` rows of C and all columns of C, so each element
// of A is read from HBM exactly once.  The contraction range K is split into
// S chunks when the row blocks alone cannot fill the chip; the partials are
// summed afterwards in a fixed order (deterministic, no atomics).  Workgroup b
// takes K chunk b % S: consecutive workgroups land on different XCDs, so the
// workgroups sharing one chunk of X run on the same XCD(s) and read it from
// their own L2.
//
// Tiles are staged through LDS: a stage of A (bm x bk or bk x bm) is loaded
// with 16-byte coalesced loads into registers while the previous stage is
// multiplied, then written to LDS; X is staged alongside.
//
//   FP32  : v_mfma_f32_32x32x2f32, 4 waves x 32 rows, bk = 32.
//   FP64  : v_mfma_f64_16x16x4f64, 4 waves x 16 rows, bk = 16.
//   BF16  : v_mfma_f32_32x32x16_bf16, 4 waves x 32 rows, bk = 32.  A and X
//           are split on the fly into bfloat16 a_hi = rn(a), a_lo = rn(a - a_hi);
//           bf16x3 accumulates a_hi b_hi + a_hi b_lo + a_lo b_hi in FP32, plain
//           BF16 only a_hi b_hi.
#include "common.hpp"

namespace rsvd {

namespace {

template <typename T>
__device__ inline void load_run4(const T* base, int valid, bool vec, T out[4]);

template <>
__device__ inline void load_run4<float>(const float* base, int valid, bool vec, float out[4]) {
  if (valid == 4 && vec) {
    const f32x4 v = *reinterpret_cast<const f32x4*>(base);
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2];
    out[3] = v[3];
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e] = (e < valid) ? base[e] : 0.f;
  }
}

template <>
__device__ inline void load_run4<double>(const double* base, int valid, bool vec, double out[4]) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  if (valid == 4 && vec) {
    const d2 v0 = *reinterpret_cast<const d2*>(base);
    const d2 v1 = *reinterpret_cast<const d2*>(base + 2);
    out[0] = v0[0];
    out[1] = v0[1];
    out[2] = v1[0];
    out[3] = v1[1];
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e] = (e < valid) ? base[e] : 0.0;
  }
}

__device__ inline int clamp_valid(int64_t v) { return v <= 0 ? 0 : (v >= 4 ? 4 : (int)v); }

// Loads of one stage into registers, shared by the three variants.  A stage of
// A is BM x BK (NN) or BK x BM (TN) elements, NRUN runs of four per thread;
// X is BK x 128 elements, NX per thread.
template <typename T, bool TRANS, int BM, int BK, int NRUN>
__device__ inline void stage_load_a(const GemmParams& p, int64_t i0, int64_t k0, int64_t kend, int tid,
                                    T (&ra)[NRUN * 4]) {
  const T* A = (const T*)p.A;  // may alias p.out (in-place Y R^-1): not restrict
  constexpr int RUNS_PER_ROW = TRANS ? BM / 4 : BK / 4;  // runs along the contiguous dimension
  constexpr int ROWS_PER_PASS = 256 / RUNS_PER_ROW;
#pragma unroll
  for (int it = 0; it < NRUN; ++it) {
    const int rr = tid / RUNS_PER_ROW + ROWS_PER_PASS * it;
    const int cc = 4 * (tid % RUNS_PER_ROW);
    int valid;
    int64_t off;
    if (!TRANS) {
      const int64_t row = i0 + rr;
      const int64_t kc = k0 + cc;
      valid = row < p.rows ? clamp_valid(kend - kc) : 0;
      off = row * p.lda + kc;
    } else {
      const int64_t kr = k0 + rr;
      const int64_t col = i0 + cc;
      valid = kr < kend ? clamp_valid(p.rows - col) : 0;
      off = kr * p.lda + col;
    }
    T v[4];
    load_run4<T>(A + (valid > 0 ? off : 0), valid, p.vec != 0, v);
#pragma unroll
    for (int e = 0; e < 4; ++e) ra[4 * it + e] = v[e];
  }
}

template <typename T, int BK, int NX>
__device__ inline void stage_load_x(const GemmParams& p, int64_t k0, int64_t kend, int tid, T (&rx)[NX]) {
  const T* __restrict__ X = (const T*)p.X;
#pragma unroll
  for (int it = 0; it < NX; ++it) {
    const int idx = tid + 256 * it;
    const int kr = idx >> 7;
    const int c = idx & 127;
    const int64_t kk = k0 + kr;
    rx[it] = (kk < kend && c < p.ncols) ? X[kk * p.ldx + c] : (T)0;
  }
}

// ---------------------------------------------------------------------------
// FP32: v_mfma_f32_32x32x2f32.  Operand lanes: A[i = lane%32][k = lane/32],
// B[k = lane/32][j = lane%32]; result register e of lane holds
// C[8*(e/4) + 4*(lane/32) + e%4][lane%32].
//
// Two row-block sizes: 128 rows (each wave 32 rows x all columns), and 32 rows
// (each wave one 32-column tile of the same 32 rows) when the caller asks for
// it on a short contraction, so that one small product such as Y R^-1 spreads
// over four times as many workgroups (a batch of products fills the chip
// without it).  Either way a workgroup reads all of its rows of
// A before it writes any row of C (in-place Y R^-1 stays safe).
__host__ __device__ inline int f32_block_rows(const GemmParams& p) { return (p.narrow && p.S == 1 && p.K <= 256) ? 32 : 128; }

// LDS row strides of the stages: an MFMA operand read takes 32 consecutive
// elements from each of two rows (one per half-wave), so a stride of 32
// modulo the 64 banks puts the halves on disjoint banks.
constexpr int F32_BK = 32;
constexpr int F32_AS = F32_BK * (128 + 32);  // LDS floats of the A stage (largest layout)
constexpr int F32_XLD = 128 + 32;

template <bool TRANS, int BM>
__device__ __forceinline__ void gemm_f32_body(const GemmParams& p, const int bid, float* As, float* Xs) {
  constexpr int BK = F32_BK;
  constexpr int ALD = TRANS ? (BM % 64 == 32 ? BM : BM + 32) : BK + 1;
  constexpr int XLD = F32_XLD;
  static_assert(XLD % 64 == 32 && (!TRANS || ALD % 64 == 32), "stage strides off the bank pattern");
  constexpr int NRUN = BM * BK / 1024;  // runs of four A elements per thread and stage
  constexpr int RUNS_PER_ROW = TRANS ? BM / 4 : BK / 4;
  constexpr int ROWS_PER_PASS = 256 / RUNS_PER_ROW;
  static_assert(TRANS ? BK * ALD <= F32_AS : BM * ALD <= F32_AS, "A stage exceeds its LDS");
  if (p.gate && *p.gate == 0) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int S = p.S;
  const int s = bid % S;
  const int64_t i0 = (int64_t)(bid / S) * BM;
  const int64_t kbeg = (int64_t)s * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int NT = p.Lp / 32;
  const int rbase = BM == 128 ? wave * 32 : 0;  // first row of this wave's tiles

  f32x16 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x16{};

  float ra[NRUN * 4], rx[16];
  const int64_t nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    stage_load_a<float, TRANS, BM, BK, NRUN>(p, i0, kbeg, kend, tid, ra);
    stage_load_x<float, BK, 16>(p, kbeg, kend, tid, rx);
  }
  const int r = lane & 31, g = lane >> 5;
  for (int64_t kt = 0; kt < nk; ++kt) {
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NRUN; ++it) {
      const int rr = tid / RUNS_PER_ROW + ROWS_PER_PASS * it, cc = 4 * (tid % RUNS_PER_ROW);
      if (!TRANS) {
#pragma unroll
        for (int e = 0; e < 4; ++e) As[rr * ALD + cc + e] = ra[4 * it + e];
      } else {
        *reinterpret_cast<f32x4*>(&As[rr * ALD + cc]) =
            f32x4{ra[4 * it], ra[4 * it + 1], ra[4 * it + 2], ra[4 * it + 3]};
      }
    }
#pragma unroll
    for (int it = 0; it < 16; ++it) {
      const int idx = tid + 256 * it;
      Xs[(idx >> 7) * XLD + (idx & 127)] = rx[it];
    }
    __syncthreads();
    if (kt + 1 < nk) {
      const int64_t k0 = kbeg + (kt + 1) * BK;
      stage_load_a<float, TRANS, BM, BK, NRUN>(p, i0, k0, kend, tid, ra);
      stage_load_x<float, BK, 16>(p, k0, kend, tid, rx);
    }
#pragma unroll
    for (int ks = 0; ks < BK / 2; ++ks) {
      const int kl = 2 * ks + g;
      const float a = TRANS ? As[kl * ALD + rbase + r] : As[(rbase + r) * ALD + kl];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (BM == 128 ? t < NT : (t == wave && t < NT)) {
          const float b = Xs[kl * XLD + t * 32 + r];
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[t], 0, 0, 0);
        }
      }
    }
  }

  float* out = (float*)p.out;
  float* part = (float*)p.part;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (t >= NT || (BM == 32 && t != wave)) continue;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int64_t row = i0 + rbase + 8 * (e >> 2) + 4 * g + (e & 3);
      const int col = t * 32 + r;
      if (row < p.rows) {
        if (S == 1) {
          if (col < p.ncols) {
            const int64_t o = row * p.ldo + col;
            out[o] = p.accum ? out[o] + acc[t][e] : acc[t][e];
          }
        } else {
          part[((int64_t)s * p.rows + row) * p.Lp + col] = acc[t][e];
        }
      }
    }
  }
}

template <bool TRANS>
__device__ __forceinline__ void gemm_f32_any(const GemmParams& p, const int bid) {
  __shared__ __attribute__((aligned(16))) float As[F32_AS];
  __shared__ __attribute__((aligned(16))) float Xs[F32_BK * F32_XLD];
  if (f32_block_rows(p) == 32)
    gemm_f32_body<TRANS, 32>(p, bid, As, Xs);
  else
    gemm_f32_body<TRANS, 128>(p, bid, As, Xs);
}

template <bool TRANS>
__global__ __launch_bounds__(256, 2) void gemm_f32_kernel(const GemmParams p) { gemm_f32_any<TRANS>(p, blockIdx.x); }

template <bool TRANS>
__global__ __launch_bounds__(256, 2) void gemm_f32_batched(const GemmParams* __restrict__ ps, const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  gemm_f32_any<TRANS>(ps[b.item], b.local);
}

// FP32, one short product (C = A X with K <= 128, the 32-row blocks above):
// all of K is loaded into registers at once, so the global-load latency is
// exposed once rather than once per K stage.  Each wave computes one 32 x 32
// tile of the block; the MFMA's two k slots take the two halves of K (lane
// half g holds k in [g Kh, g Kh + Kh), Kh = ceil(K / 2)), so a lane's A values
// are a contiguous run of its row.  Two accumulators break the chain of
// dependent MFMAs.  A may alias C (in-place Y R^-1): every wave has consumed
// its loads before the barrier that precedes the first store.
__host__ __device__ inline bool f32_direct(bool trans, const GemmParams& p) {
  return !trans && f32_block_rows(p) == 32 && p.K <= 128;
}

template <int KH>  // K <= 2 KH; every lane issues 2 KH loads and KH MFMAs whatever K is
__global__ __launch_bounds__(256, 2) void gemm_f32_direct_kernel(const GemmParams p) {
  if (p.gate && *p.gate == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, t = tid >> 6;
  const int r = lane & 31, g = lane >> 5;
  const int64_t i0 = (int64_t)blockIdx.x * 32;
  const int64_t row = i0 + r;
  const int K = (int)p.K;
  const int Kh = (K + 1) >> 1;
  const int kb = g * Kh;
  const int col = 32 * t + r;
  const float* A = (const float*)p.A;  // may alias p.out: not restrict
  const float* X = (const float*)p.X;
  f32x16 acc0 = f32x16{}, acc1 = f32x16{};
  if (32 * t < p.ncols) {
    // Branch-free loads, all issued before the first MFMA waits on them:
    // indices are clamped into the operands and A's values past this half's
    // K are scaled by zero (a multiply keeps every load live, where a select
    // on the uniform bound would become a branch with a wait per load).  X
    // past K needs no mask: its A factor is zero and its value a finite
    // element of X.  Rows past p.rows read the last row; their results are
    // never stored.
    float a[KH], b[KH];
    const int64_t rowc = row < p.rows ? row : p.rows - 1;
    const int colc = col < p.ncols ? col : p.ncols - 1;
    if (p.vec != 0 && K % 8 == 0) {  // 16-byte runs of the row: kb + s is a multiple of 4 below Kh
#pragma unroll
      for (int s = 0; s < KH; s += 4) {
        const int sc = s < Kh ? s : 0;
        const float m = s < Kh ? 1.f : 0.f;
        const f32x4 v = *reinterpret_cast<const f32x4*>(A + rowc * p.lda + kb + sc);
#pragma unroll
        for (int e = 0; e < 4; ++e) a[s + e] = v[e] * m;
      }
    } else {
#pragma unroll
      for (int s = 0; s < KH; ++s) {
        const int k = kb + s;
        const float m = (s < Kh && k < K) ? 1.f : 0.f;
        a[s] = A[rowc * p.lda + (k < K ? k : K - 1)] * m;
      }
    }
#pragma unroll
    for (int s = 0; s < KH; ++s) {
      const int k = kb + s;
      b[s] = X[(int64_t)(k < K ? k : K - 1) * p.ldx + colc];
    }
#pragma unroll
    for (int s = 0; s < KH; s += 2) {
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], b[s], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s + 1], b[s + 1], acc1, 0, 0, 0);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);  // this wave's loads have returned
  __syncthreads();
  if (32 * t >= p.ncols || col >= p.ncols) return;
  float* out = (float*)p.out;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int64_t ro = i0 + 8 * (e >> 2) + 4 * g + (e & 3);
    if (ro < p.rows) {
      const int64_t o = ro * p.ldo + col;
      const float v = acc0[e] + acc1[e];
      out[o] = p.accum ? out[o] + v : v;
    }
  }
}

// ---------------------------------------------------------------------------
// FP64: v_mfma_f64_16x16x4f64.  Operand lanes: A[i = lane%16][k = lane/16],
// B[k = lane/16][j = lane%16]; result register e of lane holds
// C[4*e + lane/16][lane%16].
template <bool TRANS>
__device__ __forceinline__ void gemm_f64_body(const GemmParams& p, const int bid) {
  constexpr int BM = 64, BK = 16;
  constexpr int ALD = TRANS ? BM + 2 : BK + 1;
  constexpr int XLD = 128 + 2;
  __shared__ __attribute__((aligned(16))) double As[TRANS ? BK * (BM + 2) : BM * (BK + 1)];
  __shared__ __attribute__((aligned(16))) double Xs[BK * XLD];
  if (p.gate && *p.gate == 0) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int S = p.S;
  const int s = bid % S;
  const int64_t i0 = (int64_t)(bid / S) * BM;
  const int64_t kbeg = (int64_t)s * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int NT = p.Lp / 16;

  f64x4 acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = f64x4{};

  double ra[4], rx[8];
  const int64_t nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    stage_load_a<double, TRANS, BM, BK, 1>(p, i0, kbeg, kend, tid, ra);
    stage_load_x<double, BK, 8>(p, kbeg, kend, tid, rx);
  }
  const int r = lane & 15, g = lane >> 4;
  for (int64_t kt = 0; kt < nk; ++kt) {
    __syncthreads();
    if (!TRANS) {
      const int rr = tid >> 2, cc = 4 * (tid & 3);
#pragma unroll
      for (int e = 0; e < 4; ++e) As[rr * ALD + cc + e] = ra[e];
    } else {
      const int rr = tid >> 4, cc = 4 * (tid & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) As[rr * ALD + cc + e] = ra[e];
    }
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int idx = tid + 256 * it;
      Xs[(idx >> 7) * XLD + (idx & 127)] = rx[it];
    }
    __syncthreads();
    if (kt + 1 < nk) {
      const int64_t k0 = kbeg + (kt + 1) * BK;
      stage_load_a<double, TRANS, BM, BK, 1>(p, i0, k0, kend, tid, ra);
      stage_load_x<double, BK, 8>(p, k0, kend, tid, rx);
    }
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kl = 4 * ks + g;
      const double a = TRANS ? As[kl * ALD + wave * 16 + r] : As[(wave * 16 + r) * ALD + kl];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if (t < NT) {
          const double b = Xs[kl * XLD + t * 16 + r];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
        }
      }
    }
  }

  double* out = (double*)p.out;
  double* part = (double*)p.part;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    if (t >= NT) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t row = i0 + wave * 16 + 4 * e + g;
      const int col = t * 16 + r;
      if (row < p.rows) {
        if (S == 1) {
          if (col < p.ncols) {
            const int64_t o = row * p.ldo + col;
            out[o] = p.accum ? out[o] + acc[t][e] : acc[t][e];
          }
        } else {
          part[((int64_t)s * p.rows + row) * p.Lp + col] = acc[t][e];
        }
      }
    }
  }
}

template <bool TRANS>
__global__ __launch_bounds__(256, 2) void gemm_f64_kernel(const GemmParams p) { gemm_f64_body<TRANS>(p, blockIdx.x); }

// FP64 products of at most 128 x 128 x 128 (the l x l factors of the
// small-matrix steps): one wave per 16 x 16 tile of the output, operands read
// straight from memory (they sit in L2), K in steps of 4 in increasing order
// -- the order of gemm_f64_body, so the sums round the same way.
constexpr int SMALL_F64_MAX = 128;
template <bool TRANS>
__global__ __launch_bounds__(64) void gemm_f64_small_kernel(const GemmParams p) {
  if (p.gate && *p.gate == 0) return;
  const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
  const int64_t i = (int64_t)blockIdx.x * 16 + r;  // row of op(A) this lane feeds
  const int j = (int)blockIdx.y * 16 + r;          // column of X this lane feeds
  const int K = (int)p.K;
  const bool iok = i < p.rows, jok = j < p.ncols;
  const int64_t ic = iok ? i : p.rows - 1;
  const int jc = jok ? j : p.ncols - 1;
  const double* __restrict__ a = (const double*)p.A;
  const double* __restrict__ x = (const double*)p.X;
  // every load is issued unconditionally (indices clamped, values past K zeroed): a guard on the
  // runtime bound would make the compiler branch around each load and wait after it.  The steps
  // past K add exact zeros.
  double av[SMALL_F64_MAX / 4], xv[SMALL_F64_MAX / 4];
#pragma unroll
  for (int t = 0; t < SMALL_F64_MAX / 4; ++t) {
    const int k = 4 * t + g;
    const bool kok = k < K;
    const int64_t kc = kok ? k : K - 1;
    const double va = TRANS ? a[kc * p.lda + ic] : a[ic * p.lda + kc];
    const double vx = x[kc * p.ldx + jc];
    av[t] = (kok && iok) ? va : 0.0;
    xv[t] = (kok && jok) ? vx : 0.0;
  }
  const int nk = (K + 3) / 4;
  f64x4 acc{};
#pragma unroll
  for (int t = 0; t < SMALL_F64_MAX / 4; ++t) {
    const f64x4 nxt = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], xv[t], acc, 0, 0, 0);
    acc = t < nk ? nxt : acc;
  }
  double* out = (double*)p.out;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t row = (int64_t)blockIdx.x * 16 + 4 * e + g;
    if (row < p.rows && jok) {
      const int64_t o = row * p.ldo + j;
      out[o] = p.accum ? out[o] + acc[e] : acc[e];
    }
  }
}

template <bool TRANS>
__global__ __launch_bounds__(256, 2) void gemm_f64_batched(const GemmParams* __restrict__ ps, const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  gemm_f64_body<TRANS>(ps[b.item], b.local);
}

// ---------------------------------------------------------------------------
// BF16 / bf16x3: v_mfma_f32_32x32x16_bf16.  Operand lanes: A[i = lane%32][k =
// 8*(lane/32) + t], B[k = 8*(lane/32) + t][j = lane%32] for t = 0..7; result
// layout as the FP32 32x32 instruction.  A stays FP32 in LDS and is split when
// its fragment is read (each element is read by one wave once); X is split
// once per stage into transposed hi/lo planes so a B fragment is one 16-byte
// LDS read.
template <bool TRANS, int NP>
__device__ __forceinline__ void gemm_bf16_body(const GemmParams& p, const int bid) {
  constexpr int BM = 128, BK = 32;
  constexpr int ALD = TRANS ? BM + 4 : BK + 4;
  constexpr int XT = BK + 8;  // bf16 elements per transposed X column
  __shared__ __attribute__((aligned(16))) float As[TRANS ? BK * (BM + 4) : BM * (BK + 4)];
  __shared__ __attribute__((aligned(16))) __bf16 Xh[128 * XT];
  __shared__ __attribute__((aligned(16))) __bf16 Xl[NP == 3 ? 128 * XT : 8];
  if (p.gate && *p.gate == 0) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int S = p.S;
  const int s = bid % S;
  const int64_t i0 = (int64_t)(bid / S) * BM;
  const int64_t kbeg = (int64_t)s * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int NT = p.Lp / 32;

  f32x16 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x16{};

  float ra[16], rx[16];
  const int64_t nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    stage_load_a<float, TRANS, BM, BK, 4>(p, i0, kbeg, kend, tid, ra);
    stage_load_x<float, BK, 16>(p, kbeg, kend, tid, rx);
  }
  const int r = lane & 31, g = lane >> 5;
  for (int64_t kt = 0; kt < nk; ++kt) {
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      int rr, cc;
      if (!TRANS) {
        rr = (tid >> 3) + 32 * it;
        cc = 4 * (tid & 7);
      } else {
        rr = (tid >> 5) + 8 * it;
        cc = 4 * (tid & 31);
      }
      *reinterpret_cast<f32x4*>(&As[rr * ALD + cc]) =
          f32x4{ra[4 * it], ra[4 * it + 1], ra[4 * it + 2], ra[4 * it + 3]};
    }
#pragma unroll
    for (int it = 0; it < 16; ++it) {
      const int idx = tid + 256 * it;
      const int kr = idx >> 7, c = idx & 127;
      const __bf16 hi = (__bf16)rx[it];
      Xh[c * XT + kr] = hi;
      if (NP == 3) Xl[c * XT + kr] = (__bf16)(rx[it] - (float)hi);
    }
    __syncthreads();
    if (kt + 1 < nk) {
      const int64_t k0 = kbeg + (kt + 1) * BK;
      stage_load_a<float, TRANS, BM, BK, 4>(p, i0, k0, kend, tid, ra);
      stage_load_x<float, BK, 16>(p, k0, kend, tid, rx);
    }
#pragma unroll
    for (int ks = 0; ks < BK / 16; ++ks) {
      const int kb = 16 * ks + 8 * g;
      float av[8];
      if (!TRANS) {
        const f32x4 v0 = *reinterpret_cast<const f32x4*>(&As[(wave * 32 + r) * ALD + kb]);
        const f32x4 v1 = *reinterpret_cast<const f32x4*>(&As[(wave * 32 + r) * ALD + kb + 4]);
        av[0] = v0[0]; av[1] = v0[1]; av[2] = v0[2]; av[3] = v0[3];
        av[4] = v1[0]; av[5] = v1[1]; av[6] = v1[2]; av[7] = v1[3];
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) av[t] = As[(kb + t) * ALD + wave * 32 + r];
      }
      bf16x8 ahi, alo;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        ahi[t] = (__bf16)av[t];
        if (NP == 3) alo[t] = (__bf16)(av[t] - (float)ahi[t]);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < NT) {
          const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(&Xh[(t * 32 + r) * XT + kb]);
          if (NP == 3) {
            const bf16x8 blo = *reinterpret_cast<const bf16x8*>(&Xl[(t * 32 + r) * XT + kb]);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bhi, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, blo, acc[t], 0, 0, 0);
          }
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bhi, acc[t], 0, 0, 0);
        }
      }
    }
  }

  float* out = (float*)p.out;
  float* part = (float*)p.part;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (t >= NT) continue;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int64_t row = i0 + wave * 32 + 8 * (e >> 2) + 4 * g + (e & 3);
      const int col = t * 32 + r;
      if (row < p.rows) {
        if (S == 1) {
          if (col < p.ncols) {
            const int64_t o = row * p.ldo + col;
            out[o] = p.accum ? out[o] + acc[t][e] : acc[t][e];
          }
        } else {
          part[((int64_t)s * p.rows + row) * p.Lp + col] = acc[t][e];
        }
      }
    }
  }
}

template <bool TRANS, int NP>
__global__ __launch_bounds__(256, 2) void gemm_bf16_kernel(const GemmParams p) { gemm_bf16_body<TRANS, NP>(p, blockIdx.x); }

template <bool TRANS, int NP>
__global__ __launch_bounds__(256, 2) void gemm_bf16_batched(const GemmParams* __restrict__ ps, const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  gemm_bf16_body<TRANS, NP>(ps[b.item], b.local);
}

}  // namespace

GemmTile gemm_tile(int dtype, int prec) {
  if (dtype == RSVD_F64) return GemmTile{64, 16, 16};
  (void)prec;
  return GemmTile{128, 32, 32};
}

int64_t gemm_blocks(int dtype, int prec, const GemmParams& p) {
  const GemmTile tile = gemm_tile(dtype, prec);
  const int bm = (dtype == RSVD_F32 && prec == PREC_NATIVE) ? f32_block_rows(p) : tile.bm;
  return (p.rows + bm - 1) / bm * p.S;
}

namespace {

bool gemm_params_ok(int dtype, int prec, const GemmParams& p) {
  const GemmTile tile = gemm_tile(dtype, prec);
  return p.ncols <= 128 && p.Lp <= 128 && p.Lp % tile.lp_mult == 0 && p.Lp >= p.ncols && p.S >= 1 &&
         !(p.accum && p.S > 1);
}

}  // namespace

hipError_t launch_gemm(int dtype, int prec, bool trans, const GemmParams& p, hipStream_t st) {
  if (p.rows <= 0) return hipSuccess;
  if (!gemm_params_ok(dtype, prec, p)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)gemm_blocks(dtype, prec, p)), block(256);
  const bool small_f64 =
      p.S == 1 && p.rows <= SMALL_F64_MAX && p.K <= SMALL_F64_MAX && p.K >= 1 && p.ncols >= 1;
  if (dtype == RSVD_F64 && small_f64) {
    const dim3 gs((unsigned)((p.rows + 15) / 16), (unsigned)((p.ncols + 15) / 16));
    if (trans)
      hipLaunchKernelGGL(gemm_f64_small_kernel<true>, gs, dim3(64), 0, st, p);
    else
      hipLaunchKernelGGL(gemm_f64_small_kernel<false>, gs, dim3(64), 0, st, p);
  } else if (dtype == RSVD_F64) {
    if (trans)
      hipLaunchKernelGGL(gemm_f64_kernel<true>, grid, block, 0, st, p);
    else
      hipLaunchKernelGGL(gemm_f64_kernel<false>, grid, block, 0, st, p);
  } else if (prec == PREC_BF16X3) {
    if (trans)
      hipLaunchKernelGGL((gemm_bf16_kernel<true, 3>), grid, block, 0, st, p);
    else
      hipLaunchKernelGGL((gemm_bf16_kernel<false, 3>), grid, block, 0, st, p);
  } else if (prec == PREC_BF16) {
    if (trans)
      hipLaunchKernelGGL((gemm_bf16_kernel<true, 1>), grid, block, 0, st, p);
    else
      hipLaunchKernelGGL((gemm_bf16_kernel<false, 1>), grid, block, 0, st, p);
  } else if (f32_direct(trans, p)) {
    if (p.K <= 32)
      hipLaunchKernelGGL(gemm_f32_direct_kernel<16>, grid, block, 0, st, p);
    else if (p.K <= 64)
      hipLaunchKernelGGL(gemm_f32_direct_kernel<32>, grid, block, 0, st, p);
    else
      hipLaunchKernelGGL(gemm_f32_direct_kernel<64>, grid, block, 0, st, p);
  } else {
    if (trans)
      hipLaunchKernelGGL(gemm_f32_kernel<true>, grid, block, 0, st, p);
    else
      hipLaunchKernelGGL(gemm_f32_kernel<false>, grid, block, 0, st, p);
  }
  return hipGetLastError();
}

hipError_t launch_gemm_batched(int dtype, int prec, bool trans, const GemmParams* ps, const BlockMap* bm,
                               int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)nblocks), block(256);
  if (dtype == RSVD_F64) {
    if (trans)
      hipLaunchKernelGGL(gemm_f64_batched<true>, grid, block, 0, st, ps, bm);
    else
      hipLaunchKernelGGL(gemm_f64_batched<false>, grid, block, 0, st, ps, bm);
  } else if (prec == PREC_BF16X3) {
    if (trans)
      hipLaunchKernelGGL((gemm_bf16_batched<true, 3>), grid, block, 0, st, ps, bm);
    else
      hipLaunchKernelGGL((gemm_bf16_batched<false, 3>), grid, block, 0, st, ps, bm);
  } else if (prec == PREC_BF16) {
    if (trans)
      hipLaunchKernelGGL((gemm_bf16_batched<true, 1>), grid, block, 0, st, ps, bm);
    else
      hipLaunchKernelGGL((gemm_bf16_batched<false, 1>), grid, block, 0, st, ps, bm);
  } else {
    if (trans)
      hipLaunchKernelGGL(gemm_f32_batched<true>, grid, block, 0, st, ps, bm);
    else
      hipLaunchKernelGGL(gemm_f32_batched<false>, grid, block, 0, st, ps, bm);
  }
  return hipGetLastError();
}

}  // namespace rsvd
