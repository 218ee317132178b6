// The GEMMs that stream A through HBM: Y = A X (sketch and power steps,
// Algorithm 4.1 step 2, Algorithm 4.4 step 5) and Z = A^T X (power steps and
// projection, Algorithm 4.4 step 4, Algorithm 5.1 step 1), in FP32 (FP32 MFMA)
// or BF16 / bf16x3 (BF16 MFMA, FP32 accumulation).
//
// Layout of the work.  C (rows x ncols, ncols <= 128) is cut into blocks of
// 128 rows; a workgroup of two waves computes one block over one chunk of the
// contraction range, each wave a 64 x 128 tile (2 x 4 MFMA tiles of 32 x 32),
// so every A fragment feeds four MFMAs and every X fragment two.  Chunks of K
// are split across workgroups when the row blocks alone cannot fill the chip;
// workgroup b takes chunk b % S, which spreads one chunk's X over a subset of
// XCDs, and the partial products are summed afterwards in a fixed order.
//
// X is packed once per call by pack_x: zero-padded to Lp columns and a
// multiple of 32 rows, and for BF16 split into hi/lo planes stored as 32-row
// tiles with K contiguous per column -- the layout of the LDS stage -- so a
// stage of X is a straight 16-byte copy.  A is loaded with 16-byte loads into
// registers two stages ahead (enough bytes in flight per CU to cover HBM
// latency), then written to LDS: FP32 as is, BF16 split into a_hi = rn(a),
// a_lo = rn(a - a_hi) with K contiguous per row (for A^T the 4 x 4 register
// block is transposed first).  LDS is double-buffered: one barrier per stage.
#include <type_traits>

#include "common.hpp"

namespace rsvd {

namespace {

constexpr int SBM = 128;       // rows of C per workgroup
constexpr int SBK = 32;        // K per stage
constexpr int STHREADS = 128;  // two waves
constexpr int BPAD = 40;       // bf16 elements per LDS row (32 + 8 pad)

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---- pack X -----------------------------------------------------------
// One workgroup per 32-row tile of X: the tile is read with coalesced loads
// into LDS, then written as Lp columns of 32 consecutive k -- FP32 rows of Lp
// (plain) or 16-byte runs of bf16 hi and lo planes (split).
// Workgroup b packs the 32-row tile b / nch of X, columns 128 (b % nch) ..
// +127 (nch = Lp / 128 chunks when Lp > 128, else one chunk of Lp columns).
template <bool SPLIT>
__device__ __forceinline__ void pack_x_body(const GemmParams& p, const int64_t bid) {
  __shared__ float tile[32][128 + 1];
  if (p.gate && *p.gate == 0) return;
  const float* __restrict__ X = (const float*)p.X;
  const int64_t K = p.K, ldx = p.ldx, Kpad = (p.K + SBK - 1) / SBK * SBK;
  const int32_t ncols = p.ncols, Lp = p.Lp;
  const int nch = (Lp + 127) >> 7;
  const int64_t kt = bid / nch;
  const int c0 = 128 * (int)(bid - kt * nch);
  const int w = min(128, Lp - c0);  // columns of this chunk
  void* __restrict__ out = p.pack;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < 32 * w; idx += 256) {
    const int kk = idx / w, c = idx - kk * w;
    const int64_t k = kt * 32 + kk;
    tile[kk][c] = (k < K && c0 + c < ncols) ? X[k * ldx + c0 + c] : 0.f;
  }
  __syncthreads();
  if (!SPLIT) {
    float* o = (float*)out + kt * 32 * Lp + c0;
    for (int idx = tid; idx < 32 * w; idx += 256) {
      const int kk = idx / w, c = idx - kk * w;
      o[kk * Lp + c] = tile[kk][c];
    }
  } else {
    // run (c, q): k = 8 q .. 8 q + 7 of column c0 + c, 16 bytes per plane
    __bf16* hi = (__bf16*)out;
    __bf16* lo = hi + Kpad * Lp;
    for (int run = tid; run < 4 * w; run += 256) {
      const int c = run >> 2, q = run & 3;
      bf16x8 h, l;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float v = tile[8 * q + t][c];
        h[t] = (__bf16)v;
        l[t] = (__bf16)(v - (float)h[t]);
      }
      const int64_t o = (kt * Lp + c0 + c) * 32 + 8 * q;
      *reinterpret_cast<bf16x8*>(hi + o) = h;
      *reinterpret_cast<bf16x8*>(lo + o) = l;
    }
  }
}

template <bool SPLIT>
__global__ __launch_bounds__(256) void pack_x_kernel(const GemmParams p) { pack_x_body<SPLIT>(p, blockIdx.x); }

template <bool SPLIT>
__global__ __launch_bounds__(256) void pack_x_batched(const GemmParams* __restrict__ ps,
                                                      const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  const GemmParams p = ps[b.item];
  pack_x_body<SPLIT>(p, b.local);
}

__device__ inline void split4(const f32x4 v, u32x2& hi, u32x2& lo) {
  __bf16 h[4], l[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    h[e] = (__bf16)v[e];
    l[e] = (__bf16)(v[e] - (float)h[e]);
  }
  hi.x = (uint32_t)__builtin_bit_cast(uint16_t, h[0]) | ((uint32_t)__builtin_bit_cast(uint16_t, h[1]) << 16);
  hi.y = (uint32_t)__builtin_bit_cast(uint16_t, h[2]) | ((uint32_t)__builtin_bit_cast(uint16_t, h[3]) << 16);
  lo.x = (uint32_t)__builtin_bit_cast(uint16_t, l[0]) | ((uint32_t)__builtin_bit_cast(uint16_t, l[1]) << 16);
  lo.y = (uint32_t)__builtin_bit_cast(uint16_t, l[2]) | ((uint32_t)__builtin_bit_cast(uint16_t, l[3]) << 16);
}

__device__ inline f32x4 load4_guard(const float* p, int valid, bool vec) {
  if (valid == 4 && vec) return *reinterpret_cast<const f32x4*>(p);
  f32x4 v;
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = e < valid ? p[e] : 0.f;
  return v;
}

__device__ inline int valid4(int64_t v) { return v <= 0 ? 0 : (v >= 4 ? 4 : (int)v); }

// Offset (bf16 elements) of element k (0..31) of row `row` in a BF16 A plane:
// rows of BPAD elements, the four 16-byte pieces of a row permuted by
// (row >> 4) & 3.  The 8-byte stores of the transposed (A^T) stage, whose
// lanes take rows four apart, then fall on four times fewer conflicting banks;
// the 16-byte operand reads (consecutive rows) stay conflict-free.
__device__ inline int apos(int row, int k) { return row * BPAD + 8 * ((k >> 3) ^ ((row >> 4) & 3)) + (k & 7); }

// One stage of A in registers: 1024 / THR runs of four floats per thread
// (THR = 128 or 256 threads; R = THR / 8 rows or k apart).
//   NN (A rows x K): run q of thread t covers row (t / 8) + R q, k 4 (t % 8) .. +3.
//   TN (A K x rows): thread t covers the 4 x 4 block k 4 (t / 32) .. +3 (plus
//   R b for block b), columns 4 (t % 32) .. +3; run q = 4 b + r is row r of
//   block b.
template <bool TRANS, bool FAST = false, int THR = STHREADS>
__device__ inline void load_a_stage(const GemmParams& p, int64_t i0, int64_t k0, int64_t kend, int tid,
                                    f32x4 (&ra)[1024 / THR]) {
  constexpr int RUNS = 1024 / THR, RS = THR / 8;
  const float* A = (const float*)p.A;
  const bool vec = p.vec != 0;
  // FAST: a stage inside the matrix (every row / column of the block, every k
  // of the stage) with 16-byte aligned runs takes plain 16-byte loads, no
  // per-run guards.
  if (FAST && vec && i0 + SBM <= p.rows && k0 + SBK <= kend) {
#pragma unroll
    for (int q = 0; q < RUNS; ++q) {
      int64_t off;
      if (!TRANS) {
        off = (i0 + (tid >> 3) + RS * q) * p.lda + k0 + 4 * (tid & 7);
      } else {
        const int b = q >> 2, r = q & 3;
        off = (k0 + 4 * (tid >> 5) + RS * b + r) * p.lda + i0 + 4 * (tid & 31);
      }
      ra[q] = *reinterpret_cast<const f32x4*>(A + off);
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < RUNS; ++q) {
    int64_t off;
    int valid;
    if (!TRANS) {
      const int64_t row = i0 + (tid >> 3) + RS * q;
      const int64_t kc = k0 + 4 * (tid & 7);
      valid = row < p.rows ? valid4(kend - kc) : 0;
      off = row * p.lda + kc;
    } else {
      const int b = q >> 2, r = q & 3;
      const int64_t kr = k0 + 4 * (tid >> 5) + RS * b + r;
      const int64_t col = i0 + 4 * (tid & 31);
      valid = kr < kend ? valid4(p.rows - col) : 0;
      off = kr * p.lda + col;
    }
    ra[q] = load4_guard(A + (valid > 0 ? off : 0), valid, vec);
  }
}

// A stage known to lie inside the matrix with 16-byte aligned runs: plain
// 16-byte loads (the same runs as load_a_stage).  NT: the loads carry the
// non-temporal hint (A is read once per pass).  Measured on the 16384 x 8192
// power-iteration workload it helps A X with three products per element
// (145 -> 139 us) and A^T X with one (104 -> 96 us) and costs a little in the
// other two cases, so each kernel takes the faster choice.
template <bool TRANS, int THR = STHREADS, bool NT = false>
__device__ inline void load_a_full(const GemmParams& p, int64_t i0, int64_t k0, int tid, f32x4 (&ra)[1024 / THR]) {
  constexpr int RUNS = 1024 / THR, RS = THR / 8;
  const float* A = (const float*)p.A;
#pragma unroll
  for (int q = 0; q < RUNS; ++q) {
    int64_t off;
    if (!TRANS) {
      off = (i0 + (tid >> 3) + RS * q) * p.lda + k0 + 4 * (tid & 7);
    } else {
      const int b = q >> 2, r = q & 3;
      off = (k0 + 4 * (tid >> 5) + RS * b + r) * p.lda + i0 + 4 * (tid & 31);
    }
    const f32x4* src = reinterpret_cast<const f32x4*>(A + off);
    if constexpr (NT) ra[q] = __builtin_nontemporal_load(src);
    else ra[q] = *src;
  }
}

// ---- BF16 / bf16x3 ------------------------------------------------------
// MFMA v_mfma_f32_32x32x16_bf16: lane (r = lane % 32, g = lane / 32) supplies
// A[r][8 g + t] and B[8 g + t][r], t = 0..7; result register e holds
// C[8 (e / 4) + 4 g + e % 4][r].
// WIDE: C and X wider than 128 columns, one 128-column chunk per workgroup
// (the chunk index is a runtime quantity only in this variant).
// NW waves per workgroup: with 2 each wave takes 64 rows x 128 columns of the
// block (one wave per SIMD at two workgroups per CU, the LDS limit); with 4,
// 64 rows x 64 columns, so that two waves share each SIMD and hide each
// other's LDS and MFMA latencies.  Every element of C is accumulated by one
// lane in the same order either way.
template <bool TRANS, int NP, bool WIDE, int NW = 2>
__device__ __forceinline__ void stream_bf16_body(const GemmParams& p, const __bf16* __restrict__ xh,
                                                 const __bf16* __restrict__ xl, const int bid) {
  constexpr int APLANE = SBM * BPAD;  // bf16 elements per A plane per buffer
  constexpr int XPLANE = 128 * BPAD;
  __shared__ __attribute__((aligned(16))) __bf16 sAh[2][APLANE];
  __shared__ __attribute__((aligned(16))) __bf16 sAl[2][NP == 3 ? APLANE : 8];
  __shared__ __attribute__((aligned(16))) __bf16 sXh[2][XPLANE];
  __shared__ __attribute__((aligned(16))) __bf16 sXl[2][NP == 3 ? XPLANE : 8];
  if (p.gate && *p.gate == 0) return;

  constexpr int THR = 64 * NW, RUNS_A = 1024 / THR, RUNS_X = 512 / THR, TPW = 8 / NW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = NW == 2 ? wave : (wave & 1);  // 64-row half of the block
  const int wc = NW == 2 ? 0 : (wave >> 1);    // 64-column half (NW = 4)
  const int S = p.S;
  // workgroup -> (row block, 128-column chunk of C, K chunk s)
  const int nch = WIDE ? (p.Lp + 127) >> 7 : 1;
  const int s = bid % S;
  const int tb = bid / S;
  const int ch = WIDE ? tb % nch : 0;
  const int64_t i0 = (int64_t)(WIDE ? tb / nch : tb) * SBM;
  const int64_t kbeg = (int64_t)s * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int NT = WIDE ? min(4, (p.Lp - 128 * ch) >> 5) : p.Lp / 32;
  const int64_t nk = kend > kbeg ? (kend - kbeg + SBK - 1) / SBK : 0;
  if (WIDE) {  // the chunk's columns within every 32-row tile of packed X
    xh += 128 * 32 * ch;
    xl += 128 * 32 * ch;
  }

  f32x16 acc[2][TPW];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[a][t] = f32x16{};

  // Two stages of A are kept in flight (raA / raB alternate); X, which comes
  // from L2, one stage ahead.  X loads of a stage are issued before the A loads
  // of the stage after it, so writing a stage to LDS waits only for its own loads.
  f32x4 raA[RUNS_A], raB[RUNS_A];
  u32x4 rxh[RUNS_X], rxl[RUNS_X];
  // F (a std::integral_constant): every stage full and all 128 columns of X
  // present, so the per-run guards are compiled out of the steady-state loop.
  auto load_x = [&](int64_t k0, auto F) __attribute__((always_inline)) {
    const u32x4* gh = reinterpret_cast<const u32x4*>(xh + (k0 >> 5) * (int64_t)p.Lp * 32);
    const u32x4* gl = reinterpret_cast<const u32x4*>(xl + (k0 >> 5) * (int64_t)p.Lp * 32);
#pragma unroll
    for (int q = 0; q < RUNS_X; ++q) {
      const int run = tid + THR * q;
      if (decltype(F)::value || run < NT * 128) {
        rxh[q] = gh[run];
        if (NP == 3) rxl[q] = gl[run];
      }
    }
  };
  auto store_stage = [&](int buf, const f32x4 (&ra)[RUNS_A], auto F) __attribute__((always_inline)) {
    // A: split and write K-contiguous rows
    if (!TRANS) {
#pragma unroll
      for (int q = 0; q < RUNS_A; ++q) {
        const int row = (tid >> 3) + (THR / 8) * q;
        const int kc = 4 * (tid & 7);
        u32x2 h, l;
        split4(ra[q], h, l);
        *reinterpret_cast<u32x2*>(&sAh[buf][apos(row, kc)]) = h;
        if (NP == 3) *reinterpret_cast<u32x2*>(&sAl[buf][apos(row, kc)]) = l;
      }
    } else {
#pragma unroll
      for (int b = 0; b < RUNS_A / 4; ++b) {
        const int kc = 4 * (tid >> 5) + (THR / 8) * b;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = 4 * (tid & 31) + e;  // column of A = row of C
          const f32x4 v = f32x4{ra[4 * b][e], ra[4 * b + 1][e], ra[4 * b + 2][e], ra[4 * b + 3][e]};
          u32x2 h, l;
          split4(v, h, l);
          *reinterpret_cast<u32x2*>(&sAh[buf][apos(row, kc)]) = h;
          if (NP == 3) *reinterpret_cast<u32x2*>(&sAl[buf][apos(row, kc)]) = l;
        }
      }
    }
    // X: 16-byte runs, run = column * 4 + quarter
#pragma unroll
    for (int q = 0; q < RUNS_X; ++q) {
      const int run = tid + THR * q;
      if (decltype(F)::value || run < NT * 128) {
        const int c = run >> 2, part = run & 3;
        *reinterpret_cast<u32x4*>(&sXh[buf][c * BPAD + 8 * part]) = rxh[q];
        if (NP == 3) *reinterpret_cast<u32x4*>(&sXl[buf][c * BPAD + 8 * part]) = rxl[q];
      }
    }
  };
  const int r = lane & 31, g = lane >> 5;
  auto compute = [&](int buf, auto F) __attribute__((always_inline)) {
#pragma unroll
    for (int ks = 0; ks < SBK / 16; ++ks) {
      const int kb = 16 * ks + 8 * g;
      bf16x8 ah[2], al[2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const int row = wr * 64 + rt * 32 + r;
        ah[rt] = *reinterpret_cast<const bf16x8*>(&sAh[buf][apos(row, kb)]);
        if (NP == 3) al[rt] = *reinterpret_cast<const bf16x8*>(&sAl[buf][apos(row, kb)]);
      }
#pragma unroll
      for (int tt = 0; tt < TPW; ++tt) {
        const int t = wc * TPW + tt;
        if (decltype(F)::value || t < NT) {
          const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&sXh[buf][(t * 32 + r) * BPAD + kb]);
          bf16x8 bl;
          if (NP == 3) bl = *reinterpret_cast<const bf16x8*>(&sXl[buf][(t * 32 + r) * BPAD + kb]);
#pragma unroll
          for (int rt = 0; rt < 2; ++rt) {
            if (NP == 3) {
              acc[rt][tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[rt], bh, acc[rt][tt], 0, 0, 0);
              acc[rt][tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[rt], bl, acc[rt][tt], 0, 0, 0);
            }
            acc[rt][tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[rt], bh, acc[rt][tt], 0, 0, 0);
          }
        }
      }
    }
  };
  auto kofs = [&](int64_t stage) { return kbeg + stage * SBK; };

  const std::false_type G{};
  const std::true_type F{};
  if (nk > 0) load_a_stage<TRANS, true, THR>(p, i0, kofs(0), kend, tid, raA);
  if (nk > 0) load_x(kofs(0), G);
  if (nk > 1) load_a_stage<TRANS, true, THR>(p, i0, kofs(1), kend, tid, raB);
  if (nk > 0) store_stage(0, raA, G);
  __syncthreads();
  int64_t kt = 0;
  // Steady state: two stages per iteration with no branch between a stage's
  // products and the next stage's split-and-store, so the compiler can
  // interleave the VALU work with the MFMAs.
  if (NT == 4 && p.vec != 0 && i0 + SBM <= p.rows && (kend - kbeg) % SBK == 0) {
    for (; kt + 3 < nk; kt += 2) {
      load_x(kofs(kt + 1), F);
      load_a_full<TRANS, THR, (NP == 3) != TRANS>(p, i0, kofs(kt + 2), tid, raA);
      compute(0, F);
      store_stage(1, raB, F);
      __syncthreads();
      load_x(kofs(kt + 2), F);
      load_a_full<TRANS, THR, (NP == 3) != TRANS>(p, i0, kofs(kt + 3), tid, raB);
      compute(1, F);
      store_stage(0, raA, F);
      __syncthreads();
    }
  }
  for (; kt < nk; kt += 2) {
    // stage kt in buffer 0; stage kt + 1 in flight in raB
    if (kt + 1 < nk) load_x(kofs(kt + 1), G);
    if (kt + 2 < nk) load_a_stage<TRANS, true, THR>(p, i0, kofs(kt + 2), kend, tid, raA);
    compute(0, G);
    if (kt + 1 < nk) store_stage(1, raB, G);
    __syncthreads();
    if (kt + 1 >= nk) break;
    // stage kt + 1 in buffer 1; stage kt + 2 in flight in raA
    if (kt + 2 < nk) load_x(kofs(kt + 2), G);
    if (kt + 3 < nk) load_a_stage<TRANS, true, THR>(p, i0, kofs(kt + 3), kend, tid, raB);
    compute(1, G);
    if (kt + 2 < nk) store_stage(0, raA, G);
    __syncthreads();
  }

  float* out = (float*)p.out;
  float* part = (float*)p.part;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
      const int t = wc * TPW + tt;
      if (t >= NT) continue;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t row = i0 + wr * 64 + rt * 32 + 8 * (e >> 2) + 4 * g + (e & 3);
        const int col = 128 * ch + t * 32 + r;
        if (row < p.rows) {
          if (S == 1) {
            if (col < p.ncols) out[row * p.ldo + col] = acc[rt][tt][e];
          } else {
            part[((int64_t)s * p.rows + row) * p.Lp + col] = acc[rt][tt][e];
          }
        }
      }
    }
  }
}

template <bool TRANS, int NP, bool WIDE>
__global__ __launch_bounds__(STHREADS, 2) __attribute__((amdgpu_waves_per_eu(1, 1))) void stream_bf16_kernel(
    const GemmParams p, const __bf16* __restrict__ xh, const __bf16* __restrict__ xl) {
  stream_bf16_body<TRANS, NP, WIDE>(p, xh, xl, blockIdx.x);
}

// Four waves per workgroup, two per SIMD (the single-problem launches).
template <bool TRANS, int NP, bool WIDE>
__global__ __launch_bounds__(4 * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void stream_bf16_kernel4(
    const GemmParams p, const __bf16* __restrict__ xh, const __bf16* __restrict__ xl) {
  stream_bf16_body<TRANS, NP, WIDE, 4>(p, xh, xl, blockIdx.x);
}

// Batched: problem bm[b].item, its own packed X (hi plane, then lo plane) at p.pack.
template <bool TRANS, int NP, bool WIDE>
__global__ __launch_bounds__(STHREADS, 2) __attribute__((amdgpu_waves_per_eu(1, 1))) void stream_bf16_batched(
    const GemmParams* __restrict__ ps, const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  const GemmParams p = ps[b.item];
  const __bf16* xh = (const __bf16*)p.pack;
  stream_bf16_body<TRANS, NP, WIDE>(p, xh, xh + (p.K + SBK - 1) / SBK * SBK * p.Lp, b.local);
}

// ---- FP32 ---------------------------------------------------------------
// MFMA v_mfma_f32_32x32x2f32: lane (r, g) supplies A[r][g] and B[g][r]; K is
// walked two at a time (k = 2 ks + g).
template <bool TRANS>
__device__ __forceinline__ void stream_f32_body(const GemmParams& p, const float* __restrict__ xp, const int bid) {
  constexpr int ALD = TRANS ? SBM + 4 : SBK + 1;
  constexpr int ASZ = TRANS ? SBK * (SBM + 4) : SBM * (SBK + 1);
  constexpr int XLD = 128 + 4;
  __shared__ __attribute__((aligned(16))) float sA[2][ASZ];
  __shared__ __attribute__((aligned(16))) float sX[2][SBK * XLD];
  if (p.gate && *p.gate == 0) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int S = p.S;
  const int s = bid % S;
  const int64_t i0 = (int64_t)(bid / S) * SBM;
  const int64_t kbeg = (int64_t)s * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int NT = p.Lp / 32;
  const int64_t nk = kend > kbeg ? (kend - kbeg + SBK - 1) / SBK : 0;

  f32x16 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[a][t] = f32x16{};

  // Two stages of A in flight, X one stage ahead (see the BF16 kernel).
  f32x4 raA[8], raB[8];
  f32x4 rx[8];
  // X stage: 32 rows x Lp floats = 8 * Lp float4 runs
  auto load_x = [&](int64_t k0) __attribute__((always_inline)) {
    const f32x4* gx = reinterpret_cast<const f32x4*>(xp + k0 * p.Lp);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int run = tid + STHREADS * q;
      if (run < SBK * p.Lp / 4) rx[q] = gx[run];
    }
  };
  auto store_stage = [&](int buf, const f32x4 (&ra)[8]) __attribute__((always_inline)) {
    if (!TRANS) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int row = (tid >> 3) + 16 * q, kc = 4 * (tid & 7);
#pragma unroll
        for (int e = 0; e < 4; ++e) sA[buf][row * ALD + kc + e] = ra[q][e];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int b = q >> 2, rr = q & 3;
        const int kr = 4 * (tid >> 5) + 16 * b + rr, c = 4 * (tid & 31);
        *reinterpret_cast<f32x4*>(&sA[buf][kr * ALD + c]) = ra[q];
      }
    }
    const int q4 = p.Lp / 4;  // float4 runs per X row
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int run = tid + STHREADS * q;
      if (run < SBK * q4) {
        const int kr = run / q4, c = 4 * (run - kr * q4);
        *reinterpret_cast<f32x4*>(&sX[buf][kr * XLD + c]) = rx[q];
      }
    }
  };
  const int r = lane & 31, g = lane >> 5;
  auto compute = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int ks = 0; ks < SBK / 2; ++ks) {
      const int kl = 2 * ks + g;
      float a[2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const int row = wave * 64 + rt * 32 + r;
        a[rt] = TRANS ? sA[buf][kl * ALD + row] : sA[buf][row * ALD + kl];
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < NT) {
          const float b = sX[buf][kl * XLD + t * 32 + r];
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
            acc[rt][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rt], b, acc[rt][t], 0, 0, 0);
        }
      }
    }
  };
  auto kofs = [&](int64_t stage) { return kbeg + stage * SBK; };

  if (nk > 0) load_a_stage<TRANS>(p, i0, kofs(0), kend, tid, raA);
  if (nk > 0) load_x(kofs(0));
  if (nk > 1) load_a_stage<TRANS>(p, i0, kofs(1), kend, tid, raB);
  if (nk > 0) store_stage(0, raA);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; kt += 2) {
    if (kt + 1 < nk) load_x(kofs(kt + 1));
    if (kt + 2 < nk) load_a_stage<TRANS>(p, i0, kofs(kt + 2), kend, tid, raA);
    compute(0);
    if (kt + 1 < nk) store_stage(1, raB);
    __syncthreads();
    if (kt + 1 >= nk) break;
    if (kt + 2 < nk) load_x(kofs(kt + 2));
    if (kt + 3 < nk) load_a_stage<TRANS>(p, i0, kofs(kt + 3), kend, tid, raB);
    compute(1);
    if (kt + 2 < nk) store_stage(0, raA);
    __syncthreads();
  }

  float* out = (float*)p.out;
  float* part = (float*)p.part;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t >= NT) continue;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t row = i0 + wave * 64 + rt * 32 + 8 * (e >> 2) + 4 * g + (e & 3);
        const int col = t * 32 + r;
        if (row < p.rows) {
          if (S == 1) {
            if (col < p.ncols) out[row * p.ldo + col] = acc[rt][t][e];
          } else {
            part[((int64_t)s * p.rows + row) * p.Lp + col] = acc[rt][t][e];
          }
        }
      }
    }
  }
}

template <bool TRANS>
__global__ __launch_bounds__(STHREADS, 2) __attribute__((amdgpu_waves_per_eu(1, 1))) void stream_f32_kernel(
    const GemmParams p, const float* __restrict__ xp) {
  stream_f32_body<TRANS>(p, xp, blockIdx.x);
}

template <bool TRANS>
__global__ __launch_bounds__(STHREADS, 2) __attribute__((amdgpu_waves_per_eu(1, 1))) void stream_f32_batched(
    const GemmParams* __restrict__ ps, const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  const GemmParams p = ps[b.item];
  stream_f32_body<TRANS>(p, (const float*)p.pack, b.local);
}

}  // namespace

int64_t stream_pack_bytes(int64_t K, int32_t Lp) {
  const int64_t Kpad = (K + SBK - 1) / SBK * SBK;
  return Kpad * Lp * 4;  // FP32, or two BF16 planes
}

// X wider than 128 columns (BF16 kernels only) is taken in 128-column chunks.
bool stream_params_ok(int prec, const GemmParams& p) {
  const bool wide_ok = p.wide && prec != PREC_NATIVE && p.Lp % 128 == 0;
  return p.ncols >= 1 && p.Lp >= p.ncols && p.Lp % 32 == 0 && (p.Lp <= 128 || wide_ok) && p.S >= 1;
}

int64_t pack_x_blocks(const GemmParams& p) { return (p.K + SBK - 1) / SBK * ((p.Lp + 127) / 128); }

int64_t stream_gemm_blocks(const GemmParams& p) {
  return p.rows <= 0 ? 0 : (p.rows + SBM - 1) / SBM * ((p.Lp + 127) / 128) * p.S;
}

hipError_t launch_pack_x(int prec, const GemmParams& p, hipStream_t st) {
  if (!stream_params_ok(prec, p)) return hipErrorInvalidValue;
  const dim3 pgrid((unsigned)pack_x_blocks(p));
  if (prec != PREC_NATIVE)
    hipLaunchKernelGGL(pack_x_kernel<true>, pgrid, dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(pack_x_kernel<false>, pgrid, dim3(256), 0, st, p);
  return hipGetLastError();
}

namespace {

// Single problems take the four-wave workgroups (two waves per SIMD).
template <bool WIDE>
void launch_bf16_single(int prec, bool trans, const GemmParams& p, dim3 grid, const __bf16* xh, const __bf16* xl,
                        hipStream_t st) {
  const dim3 block(4 * 64);
  if (prec == PREC_BF16X3) {
    if (trans)
      hipLaunchKernelGGL((stream_bf16_kernel4<true, 3, WIDE>), grid, block, 0, st, p, xh, xl);
    else
      hipLaunchKernelGGL((stream_bf16_kernel4<false, 3, WIDE>), grid, block, 0, st, p, xh, xl);
  } else {
    if (trans)
      hipLaunchKernelGGL((stream_bf16_kernel4<true, 1, WIDE>), grid, block, 0, st, p, xh, xl);
    else
      hipLaunchKernelGGL((stream_bf16_kernel4<false, 1, WIDE>), grid, block, 0, st, p, xh, xl);
  }
}

template <bool WIDE>
void launch_bf16_batched(int prec, bool trans, const GemmParams* ps, const BlockMap* bm, dim3 grid, hipStream_t st) {
  const dim3 block(STHREADS);
  if (prec == PREC_BF16X3) {
    if (trans)
      hipLaunchKernelGGL((stream_bf16_batched<true, 3, WIDE>), grid, block, 0, st, ps, bm);
    else
      hipLaunchKernelGGL((stream_bf16_batched<false, 3, WIDE>), grid, block, 0, st, ps, bm);
  } else {
    if (trans)
      hipLaunchKernelGGL((stream_bf16_batched<true, 1, WIDE>), grid, block, 0, st, ps, bm);
    else
      hipLaunchKernelGGL((stream_bf16_batched<false, 1, WIDE>), grid, block, 0, st, ps, bm);
  }
}

}  // namespace

hipError_t launch_stream_gemm(int prec, bool trans, const GemmParams& p, hipStream_t st) {
  if (p.rows <= 0) return hipSuccess;
  if (!stream_params_ok(prec, p)) return hipErrorInvalidValue;
  const int64_t Kpad = (p.K + SBK - 1) / SBK * SBK;
  const dim3 grid((unsigned)stream_gemm_blocks(p));
  if (prec == PREC_NATIVE) {
    if (trans)
      hipLaunchKernelGGL(stream_f32_kernel<true>, grid, dim3(STHREADS), 0, st, p, (const float*)p.pack);
    else
      hipLaunchKernelGGL(stream_f32_kernel<false>, grid, dim3(STHREADS), 0, st, p, (const float*)p.pack);
    return hipGetLastError();
  }
  const __bf16* xh = (const __bf16*)p.pack;
  const __bf16* xl = xh + Kpad * p.Lp;
  if (p.wide)
    launch_bf16_single<true>(prec, trans, p, grid, xh, xl, st);
  else
    launch_bf16_single<false>(prec, trans, p, grid, xh, xl, st);
  return hipGetLastError();
}

// Batched launches (parameters checked when each problem was recorded; `wide`
// is the same for every problem of a step).
hipError_t launch_pack_x_batched(int prec, const GemmParams* ps, const BlockMap* bm, int64_t nblocks,
                                 hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (prec != PREC_NATIVE)
    hipLaunchKernelGGL(pack_x_batched<true>, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
  else
    hipLaunchKernelGGL(pack_x_batched<false>, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
  return hipGetLastError();
}

hipError_t launch_stream_gemm_batched(int prec, bool trans, bool wide, const GemmParams* ps, const BlockMap* bm,
                                      int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)nblocks);
  if (prec == PREC_NATIVE) {
    if (trans)
      hipLaunchKernelGGL(stream_f32_batched<true>, grid, dim3(STHREADS), 0, st, ps, bm);
    else
      hipLaunchKernelGGL(stream_f32_batched<false>, grid, dim3(STHREADS), 0, st, ps, bm);
  } else if (wide) {
    launch_bf16_batched<true>(prec, trans, ps, bm, grid, st);
  } else {
    launch_bf16_batched<false>(prec, trans, ps, bm, grid, st);
  }
  return hipGetLastError();
}

}  // namespace rsvd
