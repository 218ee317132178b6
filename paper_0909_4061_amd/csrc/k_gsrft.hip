// The structured test matrix built from chains of random Givens rotations
// (the remark on random Givens rotations in Section 4.6), real form:
//     Omega = D'' Theta' D' Theta (sqrt(n/l) D F_r R),
//     Theta = Pi G(1, 2; theta_1) ... G(n-1, n; theta_{n-1}),
// with D', D'' random +-1 diagonals, Pi a uniformly random permutation acting
// on a row vector as the gather (x Pi)_j = x_pi(j), and G(i, k; theta) the
// rotation that maps entries (x_i, x_k) of a row vector to
// (c x_i - s x_k, s x_i + c x_k).  The SRFT kernels supply D F_r R; this file
// applies the part in front of them, T = D'' Theta' D' Theta, to every row of
// A, into a copy of A that the SRFT kernel then reads.
//
// Draws (the generator contract, chain c = 0 for (D', Theta), c = 1 for
// (D'', Theta')): sign p from counter (p, s, 3, c), d = 1 - 2 (w0 & 1); angle j
// from counter (j, s, 4, c), theta = 2 pi u(w0); permutation key p from
// counter (p, s, 5, c), key = ((w0 >> 16) << 16) | p, pi = the indices in
// increasing key order.
//
//   gsrft_table_kernel : signs, (cos, sin) pairs and permutation keys.
//   gsrft_sort_kernel  : one workgroup per chain sorts the n keys in LDS
//                        (bitonic; n is a power of two) into pi.
//   gsrft_rows_kernel  : one row of A at a time in LDS: signs, gather, the
//                        rotation chain, for each chain in turn (512 threads).  The chain is
//                        the affine recurrence
//                            v_0 = x_0,  v_{j+1} = s_j v_j + c_j x_{j+1},
//                            out_j = c_j v_j - s_j x_{j+1},  out_{n-1} = v_{n-1}
//                        (the rotation j acts on the running value v_j and the
//                        untouched x_{j+1}); each thread composes the affine maps
//                        of its segment of S = n / 512 steps, a scan over the
//                        512 segment maps (lane shuffles within a wave, then the
//                        eight wave totals) gives every segment's starting value,
//                        and each thread then replays its segment.  The step
//                        past the end is padded with (c, s) = (1, 0), x_n = 0.
#include "common.hpp"
#include "philox.hpp"

namespace rsvd {

namespace {

constexpr double kTwoPiG = 0x1.921fb54442d18p+2;  // the double nearest 2*pi
constexpr int GSRFT_THREADS = 512;

template <typename T>
__global__ __launch_bounds__(256) void gsrft_table_kernel(GsrftTables<T> t, int64_t n, uint64_t seed, uint64_t sid) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = (int)blockIdx.y;
  if (p >= n) return;
  T* sign = c == 0 ? t.sign[0] : t.sign[1];
  T* cs = c == 0 ? t.cs[0] : t.cs[1];
  uint64_t* key = c == 0 ? t.key[0] : t.key[1];
  const Philox4 ws = philox4x64_10((uint64_t)p, sid, 3, (uint64_t)c, seed, 0);
  sign[p] = (T)(1.0 - 2.0 * (double)(ws.w[0] & 1));
  T cs0 = (T)1, cs1 = (T)0;  // the padded step past the end
  if (p < n - 1) {
    const Philox4 wa = philox4x64_10((uint64_t)p, sid, 4, (uint64_t)c, seed, 0);
    const double th = kTwoPiG * philox_uniform(wa.w[0]);
    cs0 = (T)cos(th);
    cs1 = (T)sin(th);
  }
  cs[2 * p] = cs0;
  cs[2 * p + 1] = cs1;
  const Philox4 wp = philox4x64_10((uint64_t)p, sid, 5, (uint64_t)c, seed, 0);
  key[p] = ((wp.w[0] >> 16) << 16) | (uint64_t)p;
}

// n <= GSRFT_MAX_N, a power of two
template <typename T>
__global__ __launch_bounds__(1024) void gsrft_sort_kernel(GsrftTables<T> t, int n) {
  __shared__ uint64_t buf[GSRFT_MAX_N];
  const uint64_t* key = blockIdx.x == 0 ? t.key[0] : t.key[1];
  int32_t* perm = blockIdx.x == 0 ? t.perm[0] : t.perm[1];
  const T* sign = blockIdx.x == 0 ? t.sign[0] : t.sign[1];
  T* psign = blockIdx.x == 0 ? t.psign[0] : t.psign[1];
  for (int i = threadIdx.x; i < n; i += blockDim.x) buf[i] = key[i];
  __syncthreads();
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = buf[i], b = buf[ixj];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            buf[i] = b;
            buf[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int q = (int)(buf[i] & 0xFFFFull);
    perm[i] = q;
    psign[i] = sign[q];
  }
}

// LDS position of row entry j: one pad word after every 32 entries, so that the chain's per-thread
// segments (entry t S + i for thread t) fall in different banks (unpadded, S = 32 puts every lane of
// a wave on one bank)
__device__ __forceinline__ int pidx(int j) { return j + (j >> 5); }

template <typename T> struct GVec2;
template <> struct GVec2<float> { typedef float __attribute__((ext_vector_type(2))) type; };
template <> struct GVec2<double> { typedef double __attribute__((ext_vector_type(2))) type; };

// The rotation chain of one row in LDS (see the file comment).  S steps per thread, n / S threads
// (all of them when n >= GSRFT_THREADS * S; S = 1 and n threads for n < GSRFT_THREADS).  Loads are
// branch-free (clamped indices, values masked afterwards) and issued a group at a time; the
// (cos, sin) pairs are read again for the replay rather than held (they would not fit in registers
// at S = 32).
template <typename T, int S>
__device__ __forceinline__ void rotation_chain(T* buf, const T* __restrict__ cs, const int n, T* sp, T* sq) {
  typedef typename GVec2<T>::type V;
  constexpr int G = S < 16 ? S : 16;  // steps whose (cos, sin) and x are loaded together
  const int tid = threadIdx.x;
  const int nact = n / S;
  const bool act = tid < nact;
  const int j0 = act ? tid * S : 0;
  const V* csv = reinterpret_cast<const V*>(cs) + j0;
  const T x0 = buf[0];
  // x_{j+1} of the segment's last step is the next segment's first entry (zero past the end): kept
  // in a register, since the next thread overwrites it; the others are re-read from this thread's
  // own segment, which only this thread writes
  const int jl = j0 + S;
  const T xl = buf[pidx(jl < n ? jl : n - 1)];
  const T xlast = jl < n ? xl : (T)0;
  // this segment's (cos, sin) pairs, held for both passes
  V cv[S];
#pragma unroll
  for (int i = 0; i < S; ++i) cv[i] = csv[i];
  // this segment's map v -> P v + Q
  T P = (T)1, Q = (T)0;
#pragma unroll
  for (int g = 0; g < S; g += G) {
    T x[G];
#pragma unroll
    for (int i = 0; i < G; ++i) x[i] = g + i < S - 1 ? buf[pidx(j0 + g + i + 1)] : xlast;
#pragma unroll
    for (int i = 0; i < G; ++i) {
      P = cv[g + i].y * P;
      Q = cv[g + i].y * Q + cv[g + i].x * x[i];
    }
  }
  if (!act) {  // threads past the row carry the identity map
    P = (T)1;
    Q = (T)0;
  }
  __syncthreads();  // every read of buf is done: segments may now be overwritten
  // inclusive scan of the maps over the threads, I_t = map_t o ... o map_0: within each wave by
  // lane shuffles, then across the waves through their totals
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T Pe = __shfl_up(P, off, 64), Qe = __shfl_up(Q, off, 64);
    if (lane >= off) {
      Q = P * Qe + Q;
      P = P * Pe;
    }
  }
  if (lane == 63) {
    sp[GSRFT_THREADS + wv] = P;
    sq[GSRFT_THREADS + wv] = Q;
  }
  __syncthreads();
  {
    // the waves before this one, composed in order: E = total_{wv-1} o ... o total_0
    T PE = (T)1, QE = (T)0;
    for (int w = 0; w < wv; ++w) {
      const T pw = sp[GSRFT_THREADS + w], qw = sq[GSRFT_THREADS + w];
      QE = pw * QE + qw;
      PE = pw * PE;
    }
    Q = P * QE + Q;
    P = P * PE;
  }
  sp[tid] = P;
  sq[tid] = Q;
  __syncthreads();
  if (act) {
    T v = x0;
    if (tid > 0) v = sp[tid - 1] * x0 + sq[tid - 1];
#pragma unroll
    for (int g = 0; g < S; g += G) {
      T x[G];
#pragma unroll
      for (int i = 0; i < G; ++i) x[i] = g + i < S - 1 ? buf[pidx(j0 + g + i + 1)] : xlast;
#pragma unroll
      for (int i = 0; i < G; ++i) {
        buf[pidx(j0 + g + i)] = cv[g + i].x * v - cv[g + i].y * x[i];
        v = cv[g + i].y * v + cv[g + i].x * x[i];
      }
    }
  }
  __syncthreads();
}

// Raw buffer access for the element passes: the base address and size sit in a scalar
// resource, so every element of a thread is its one offset register plus a constant (global
// addressing would hold a 64-bit address per element and table, which does not fit at S = 32).
constexpr int kGsrftBufferWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t gsrft_rsrc(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kGsrftBufferWord3);
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff, float*) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff, double*) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ int buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff, int*) {
  return (int)__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}

template <typename T>
constexpr int gsrft_lds_n() {
  return 65536 / (int)sizeof(T);  // two row buffers of 64 KB
}

template <typename T, int S>
__global__ __launch_bounds__(GSRFT_THREADS) void gsrft_rows_kernel(const T* __restrict__ A, int64_t lda, int64_t m,
                                                                  int n, GsrftTables<T> t, T* __restrict__ out) {
  constexpr int NMAX = gsrft_lds_n<T>();
  __shared__ __attribute__((aligned(16))) T b0[NMAX + NMAX / 32];
  __shared__ __attribute__((aligned(16))) T b1[NMAX + NMAX / 32];
  __shared__ T sp[2 * GSRFT_THREADS], sq[2 * GSRFT_THREADS];
  const int tid = threadIdx.x;
  // element p = tid + it * GSRFT_THREADS, it < S: for S > 1, n = S * GSRFT_THREADS exactly (n is a
  // power of two), so every p is in range; for S = 1 (n <= GSRFT_THREADS) threads past n idle.
  // Every load of a pass is issued before the first use.
  const bool live = S > 1 || tid < n;
  const int tc = S > 1 ? tid : (tid < n ? tid : n - 1);
  // passes over the row's elements go in groups of G (loads of a group issued together, a
  // scheduling barrier between groups so that the registers of one group are free for the next)
  constexpr int G = S;
  const int vo = tc * (int)sizeof(T), vi = tc * 4;  // this thread's offsets (elements p = tc + k 512)
  constexpr int ST = GSRFT_THREADS * (int)sizeof(T), SI = GSRFT_THREADS * 4;
  const int64_t nb = (int64_t)n * (int64_t)sizeof(T), ni = (int64_t)n * 4;
  const __amdgpu_buffer_rsrc_t rq1 = gsrft_rsrc(t.psign[1], nb), rp1 = gsrft_rsrc(t.perm[1], ni);
  const __amdgpu_buffer_rsrc_t rp0 = gsrft_rsrc(t.perm[0], ni), rq0 = gsrft_rsrc(t.psign[0], nb);
  for (int64_t r = blockIdx.x; r < m; r += gridDim.x) {
    const __amdgpu_buffer_rsrc_t ro = gsrft_rsrc(out + r * (int64_t)n, nb);
    {
      const __amdgpu_buffer_rsrc_t ra = gsrft_rsrc(A + r * lda, nb);
      T xa[S];
#pragma unroll
      for (int it = 0; it < S; ++it) xa[it] = buf_load(ra, vo, it * ST, (T*)nullptr);
      if (live) {
#pragma unroll
        for (int it = 0; it < S; ++it) b0[pidx(tc + it * GSRFT_THREADS)] = xa[it];
      }
    }
    __syncthreads();
    // D'' and the gather of Pi': b1[j] = d''[pi'(j)] a[pi'(j)]
#pragma unroll
    for (int g = 0; g < S; g += G) {
      int q[G];
      T d[G];
#pragma unroll
      for (int it = 0; it < G; ++it) {
        q[it] = buf_load(rp1, vi, (g + it) * SI, (int*)nullptr);
        d[it] = buf_load(rq1, vo, (g + it) * ST, (T*)nullptr);
      }
      if (live) {
#pragma unroll
        for (int it = 0; it < G; ++it) b1[pidx(tc + (g + it) * GSRFT_THREADS)] = b0[pidx(q[it])] * d[it];
      }
    }
    __syncthreads();
    rotation_chain<T, S>(b1, t.cs[1], n, sp, sq);
    // D' and the gather of Pi: b0[j] = d'[pi(j)] b1[pi(j)]
#pragma unroll
    for (int g = 0; g < S; g += G) {
      int q[G];
      T d[G];
#pragma unroll
      for (int it = 0; it < G; ++it) {
        q[it] = buf_load(rp0, vi, (g + it) * SI, (int*)nullptr);
        d[it] = buf_load(rq0, vo, (g + it) * ST, (T*)nullptr);
      }
      if (live) {
#pragma unroll
        for (int it = 0; it < G; ++it) b0[pidx(tc + (g + it) * GSRFT_THREADS)] = b1[pidx(q[it])] * d[it];
      }
    }
    __syncthreads();
    rotation_chain<T, S>(b0, t.cs[0], n, sp, sq);
    if (live) {
#pragma unroll
      for (int it = 0; it < S; ++it) buf_store(b0[pidx(tc + it * GSRFT_THREADS)], ro, vo, it * ST);
    }
    __syncthreads();
  }
}

template <typename T>
hipError_t draw_t(GsrftTables<T> t, int64_t n, uint64_t seed, uint64_t sid, hipStream_t st) {
  hipLaunchKernelGGL(gsrft_table_kernel<T>, dim3((unsigned)((n + 255) / 256), 2), dim3(256), 0, st, t, n, seed, sid);
  hipLaunchKernelGGL(gsrft_sort_kernel<T>, dim3(2), dim3(1024), 0, st, t, (int)n);
  return hipGetLastError();
}

}  // namespace

size_t gsrft_table_bytes(int64_t n, int esize) {
  // per chain: n signs, n (cos, sin) pairs, n permuted signs (element type), n keys, n permutation entries
  return 2 * (size_t)n * (4 * (size_t)esize + 8 + 4) + 64;
}

template <typename T>
GsrftTables<T> gsrft_tables(void* base, int64_t n) {
  GsrftTables<T> t;
  char* b = static_cast<char*>(base);
  for (int c = 0; c < 2; ++c) {
    t.key[c] = reinterpret_cast<uint64_t*>(b);
    b += (size_t)n * 8;
  }
  for (int c = 0; c < 2; ++c) {
    t.sign[c] = reinterpret_cast<T*>(b);
    b += (size_t)n * sizeof(T);
    t.cs[c] = reinterpret_cast<T*>(b);
    b += 2 * (size_t)n * sizeof(T);
  }
  for (int c = 0; c < 2; ++c) {
    t.psign[c] = reinterpret_cast<T*>(b);
    b += (size_t)n * sizeof(T);
  }
  for (int c = 0; c < 2; ++c) {
    t.perm[c] = reinterpret_cast<int32_t*>(b);
    b += (size_t)n * 4;
  }
  return t;
}

bool gsrft_shape_ok(int dtype, int64_t n) {
  const int64_t nmax = dtype == RSVD_F64 ? gsrft_lds_n<double>() : gsrft_lds_n<float>();
  return n >= 8 && n <= nmax && n <= GSRFT_MAX_N && (n & (n - 1)) == 0;
}

hipError_t launch_gsrft_draw(int dtype, void* tables, int64_t n, uint64_t seed, uint64_t sid, hipStream_t st) {
  if (!gsrft_shape_ok(dtype, n)) return hipErrorInvalidValue;
  if (dtype == RSVD_F64) return draw_t(gsrft_tables<double>(tables, n), n, seed, sid, st);
  return draw_t(gsrft_tables<float>(tables, n), n, seed, sid, st);
}

template <typename T, int S>
void rows_launch(const dim3 grid, const void* A, int64_t lda, int64_t m, int64_t n, void* tables, void* out,
                 hipStream_t st) {
  hipLaunchKernelGGL((gsrft_rows_kernel<T, S>), grid, dim3(GSRFT_THREADS), 0, st, (const T*)A, lda, m, (int)n,
                     gsrft_tables<T>(tables, n), (T*)out);
}

template <typename T>
void rows_dispatch(const dim3 grid, const void* A, int64_t lda, int64_t m, int64_t n, void* tables, void* out,
                   hipStream_t st) {
  // S = n / GSRFT_THREADS steps per thread (1 for small n); n <= gsrft_lds_n<T>() keeps S <= 32
  const int64_t S = n > GSRFT_THREADS ? n / GSRFT_THREADS : 1;
  switch (S) {
    case 1: rows_launch<T, 1>(grid, A, lda, m, n, tables, out, st); break;
    case 2: rows_launch<T, 2>(grid, A, lda, m, n, tables, out, st); break;
    case 4: rows_launch<T, 4>(grid, A, lda, m, n, tables, out, st); break;
    case 8: rows_launch<T, 8>(grid, A, lda, m, n, tables, out, st); break;
    case 16: rows_launch<T, 16>(grid, A, lda, m, n, tables, out, st); break;
    default:
      // FP64 rows stop at n = 8192 (S = 16): only FP32 has an S = 32 variant
      if constexpr (sizeof(T) == 4) rows_launch<T, 32>(grid, A, lda, m, n, tables, out, st);
      break;
  }
}

hipError_t launch_gsrft_rows(int dtype, const void* A, int64_t lda, int64_t m, int64_t n, void* tables, void* out,
                             hipStream_t st) {
  if (!gsrft_shape_ok(dtype, n) || lda < n || m < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(m < 512 ? m : 512));
  if (dtype == RSVD_F64)
    rows_dispatch<double>(grid, A, lda, m, n, tables, out, st);
  else
    rows_dispatch<float>(grid, A, lda, m, n, tables, out, st);
  return hipGetLastError();
}

}  // namespace rsvd
