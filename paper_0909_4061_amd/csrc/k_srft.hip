// SRFT sketch Y = A Omega with Omega = sqrt(n/l) D F_r R (Section 4.6, Algorithm
// 4.5 step 2), for real A, by one FFT per row of A D -- the full transform
// followed by sampling, the variant the remark after Algorithm 4.5 prefers.
//
// F_r is the real orthonormal Fourier basis: the unitary DFT F with each
// frequency pair (q, n - q) mixed into a cosine and a sine column, the real
// tailoring of the SRFT that Section 4.6 mentions.  With X the unnormalized
// DFT of a row x of A D, the row's entry in sampled column t (frequency
// q = R_t) is
//     X_0 / sqrt(l)               q = 0
//     X_{n/2} / sqrt(l)           q = n/2
//     sqrt(2/l) Re X_q            0 < q < n/2
//    -sqrt(2/l) Im X_{n-q}        n/2 < q < n
//
// Per row (n = 2N, N = 2^LOGN):
//   * z_j = x_{2j} + i x_{2j+1}, a complex sequence of length N, is read
//     straight from HBM (one 8- or 16-byte buffer load per complex value, the
//     next row prefetched while the current one is transformed) with the
//     signs of D applied on the fly;
//   * P passes of a radix-E Stockham FFT (the self-sorting formulation of
//     Govindaraju et al., SC'08): each thread holds one radix-E butterfly in
//     registers and the N values live in LDS between passes, with one pad
//     slot after every E values, which keeps the stride-E stores of the first
//     pass free of bank conflicts and makes every LDS access a per-thread
//     base plus a compile-time offset; the twiddles of the second pass come
//     from an LDS table laid out [r][k] (conflict-free, offsets known at
//     compile time);
//   * the last radix-F pass is pruned: only the 2l bins Z_k, Z_{N-k} the
//     sampled columns need are evaluated, one per thread, each as an F-term
//     sum whose twiddles w^r are powers of one two-level table lookup;
//   * X_k = E_k + e^{-2 pi i k / n} O_k with E_k = (Z_k + conj Z_{N-k}) / 2 and
//     O_k = (Z_k - conj Z_{N-k}) / 2i, the standard real-from-half-length
//     complex FFT identity, gives the sampled row of Y.
// Workgroups are persistent and stride over rows; the cosine table, the sign
// bits and the per-column constants are set up once per workgroup.
#include <algorithm>
#include <utility>

#include "common.hpp"

namespace rsvd {

namespace {

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename T> struct Vec2;
template <> struct Vec2<float> { typedef f32x2 type; };
template <> struct Vec2<double> { typedef f64x2 type; };

template <typename V, typename T>
__device__ __forceinline__ V make2(T x, T y) {
  V v;
  v.x = x;
  v.y = y;
  return v;
}

template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
  return make2<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// cos and sin of 2 pi a / b in double at compile time (b a power of two):
// reduce to [0, pi/2] by the symmetries of cos and sin, then Taylor series
// (16 terms: the remainder is below 1e-30 there).
struct CosSin { double c, s; };
constexpr double kPi = 3.14159265358979323846;
constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k <= 16; ++k) {
    t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    s += t;
  }
  return s;
}
constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int k = 1; k <= 16; ++k) {
    t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    s += t;
  }
  return s;
}
constexpr CosSin unit_root(int a, int b) {
  a %= b;
  double sc = 1.0, ss = 1.0;
  if (2 * a > b) {  // theta -> 2 pi - theta
    a = b - a;
    ss = -1.0;
  }
  if (4 * a > b) {  // theta -> pi - theta
    a = b / 2 - a;
    sc = -1.0;
  }
  const double x = 2.0 * kPi * (double)a / (double)b;
  return CosSin{sc * taylor_cos(x), ss * taylor_sin(x)};
}

// v * exp(-2 pi i K / R) with the trivial factors written out.
template <typename V, int R, int K>
__device__ __forceinline__ V twiddle_const(V v) {
  typedef decltype(v.x + v.x) T;
  constexpr double h = 0.70710678118654752440;
  if constexpr (K == 0) {
    return v;
  } else if constexpr (4 * K == R) {
    return make2<V>(v.y, -v.x);
  } else if constexpr (8 * K == R) {
    return make2<V>((v.x + v.y) * (T)h, (v.y - v.x) * (T)h);
  } else if constexpr (8 * K == 3 * R) {
    return make2<V>((v.y - v.x) * (T)h, -(v.x + v.y) * (T)h);
  } else {
    constexpr CosSin w = unit_root(K, R);
    const T c = (T)w.c, s = (T)(-w.s);
    return make2<V>(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

// In-register DFT of length R (forward sign), natural order in and out:
// radix-2 decimation in time, unrolled at compile time.
template <int R>
struct RegDFT {
  template <typename V>
  __device__ __forceinline__ static void run(V (&a)[R]) {
    V e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = a[2 * i];
      o[i] = a[2 * i + 1];
    }
    RegDFT<R / 2>::run(e);
    RegDFT<R / 2>::run(o);
    combine(a, e, o, std::make_integer_sequence<int, R / 2>{});
  }
  template <typename V, int... K>
  __device__ __forceinline__ static void combine(V (&a)[R], const V (&e)[R / 2], const V (&o)[R / 2],
                                                 std::integer_sequence<int, K...>) {
    (butterfly<V, K>(a, e, o), ...);
  }
  template <typename V, int K>
  __device__ __forceinline__ static void butterfly(V (&a)[R], const V (&e)[R / 2], const V (&o)[R / 2]) {
    const V t = twiddle_const<V, R, K>(o[K]);
    a[K] = e[K] + t;
    a[K + R / 2] = e[K] - t;
  }
};
template <>
struct RegDFT<1> {
  template <typename V>
  __device__ __forceinline__ static void run(V (&)[1]) {}
};

struct SrftRowParams {
  const void* A;
  int64_t lda;
  int64_t m;
  int32_t l;
  int32_t vec;         // 1: rows of A allow one aligned load per complex value
  const double* d;     // n signs (+-1)
  const int32_t* R;    // l sampled frequencies in [0, n)
  void* Y;             // m x l, row-major
};

template <typename T, int LOGN>
struct SrftGeom {
  static constexpr int N = 1 << LOGN;
  static constexpr int LOGE = LOGN >= 13 ? 5 : 4;
  static constexpr int E = 1 << LOGE;               // radix of the full passes
  static constexpr int P = (LOGN - 1) / LOGE;       // number of full passes
  static constexpr int NSF = 1 << (P * LOGE);       // sub-transform length entering the pruned pass
  static constexpr int LOGF = LOGN - P * LOGE;
  static constexpr int F = 1 << LOGF;               // radix of the pruned pass, 2..E
  static constexpr int NB = N / E;                  // butterflies per full pass
  static constexpr int THREADS = NB > 128 ? NB : 128;
  static constexpr int NPAD = N + (N >> LOGE);      // one pad slot after every E values
  static constexpr int BPT = (2 * RSVD_MAX_L + THREADS - 1) / THREADS;  // sampled bins per thread
  static constexpr int TWP = P >= 2 ? E * E : 1;     // twiddles of the second full pass, [r][k]
  static constexpr int LOGLO = (LOGN + 1) / 2;       // w_N^b = hi[b >> LOGLO] lo[b mod 2^LOGLO]
  static constexpr int NLO = 1 << LOGLO, NHI = N >> LOGLO;
  static constexpr size_t LDS = (size_t)(TWP + NLO + NHI + NPAD + 2 * RSVD_MAX_L) * 2 * sizeof(T);
  static_assert(P <= 2, "at most two full passes");
};

// Raw buffer loads: the row's base address and size live in a scalar
// resource, so the per-element offsets are a thread constant plus an SGPR.
constexpr int kBufferWord3 = 0x00020000;

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const T* row, int64_t n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(row), (short)0, (int)(n * (int64_t)sizeof(T)),
                                           kBufferWord3);
}

// One complex value: a single 8- / 16-byte load when the row allows it (VEC),
// else its two parts separately.
template <bool VEC>
__device__ __forceinline__ f32x2 load_pair(__amdgpu_buffer_rsrc_t rs, int voff, int soff, f32x2*) {
  if constexpr (VEC) {
    return __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
  } else {
    f32x2 z;
    z.x = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
    z.y = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff + 4, soff, 0));
    return z;
  }
}

template <bool VEC>
__device__ __forceinline__ f64x2 load_pair(__amdgpu_buffer_rsrc_t rs, int voff, int soff, f64x2*) {
  if constexpr (VEC) {
    return __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
  } else {
    f64x2 z;
    z.x = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
    z.y = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff + 8, soff, 0));
    return z;
  }
}

// x with its sign flipped when bit `pos` (0..31) of `word` is set: one shift
// and one three-input bit operation, x ^ ((word << (31 - pos)) & 0x80000000)
// (truth table 0x6C: the middle operand xor the AND of the outer two).
__device__ __forceinline__ uint32_t flip_bits(uint32_t x, uint32_t word, int pos) {
  return __builtin_amdgcn_bitop3_b32(word << (31 - pos), x, 0x80000000u, 0x6C);
}
__device__ __forceinline__ float flip_if(float x, uint32_t word, int pos) {
  return __builtin_bit_cast(float, flip_bits(__builtin_bit_cast(uint32_t, x), word, pos));
}
__device__ __forceinline__ double flip_if(double x, uint32_t word, int pos) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t hi = flip_bits((uint32_t)(b >> 32), word, pos);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | (b & 0xffffffffull));
}

// w^r for r = 1..F-1 from w^1, each by one complex product of two earlier
// powers (squaring at powers of two), so no power is more than log2(r) + 1
// products deep.
template <int F, typename V>
__device__ __forceinline__ void unit_powers(V (&w)[F], V w1) {
  w[1] = w1;
#pragma unroll
  for (int r = 2; r < F; ++r) {
    const int hb = 1 << (31 - __builtin_clz(r));  // highest power of two <= r
    w[r] = hb == r ? cmul(w[r / 2], w[r / 2]) : cmul(w[hb], w[r - hb]);
  }
}

template <typename T, int LOGN, bool VEC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void srft_rows_kernel(SrftRowParams p) {
  typedef typename Vec2<T>::type V;
  typedef SrftGeom<T, LOGN> G;
  constexpr int N = G::N, E = G::E, LOGE = G::LOGE, P = G::P, NSF = G::NSF, F = G::F, NB = G::NB,
                THREADS = G::THREADS, BPT = G::BPT;
  constexpr int SW = (2 * E + 31) / 32;  // sign words per thread
  __shared__ V twp[G::TWP];              // twp[r * E + k] = w_{E^2}^{r k}
  __shared__ V tlo[G::NLO];              // w_N^j, j < NLO
  __shared__ V thi[G::NHI];              // w_N^{j NLO}, j < NHI
  __shared__ V data[G::NPAD];            // the row's N values, padded
  __shared__ V zbuf[2 * RSVD_MAX_L];     // the sampled bins Z_k (first l) and Z_{N-k} (next l)
  const int tid = threadIdx.x;
  const int l = p.l;

  if constexpr (P >= 2) {
    for (int j = tid; j < E * E; j += THREADS) {
      double sv, cv;
      sincospi(2.0 * (double)((j / E) * (j % E)) / (double)(E * E), &sv, &cv);
      twp[j] = make2<V>((T)cv, (T)(-sv));
    }
  }
  for (int j = tid; j < G::NLO; j += THREADS) {
    double sv, cv;
    sincospi(2.0 * (double)j / (double)N, &sv, &cv);
    tlo[j] = make2<V>((T)cv, (T)(-sv));
  }
  for (int j = tid; j < G::NHI; j += THREADS) {
    double sv, cv;
    sincospi(2.0 * (double)(j * G::NLO) / (double)N, &sv, &cv);
    thi[j] = make2<V>((T)cv, (T)(-sv));
  }

  // Signs of D for the 2E real entries this thread loads in the first pass:
  // bit 2r (real part) and 2r+1 (imaginary part) of its r-th complex value.
  uint32_t sw[SW];
#pragma unroll
  for (int w = 0; w < SW; ++w) sw[w] = 0;
  if constexpr (P >= 1) {
    if (tid < NB) {
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int c = tid + r * NB;
        const int b0 = 2 * r, b1 = 2 * r + 1;
        sw[b0 >> 5] |= (uint32_t)(p.d[2 * c] < 0.0) << (b0 & 31);
        sw[b1 >> 5] |= (uint32_t)(p.d[2 * c + 1] < 0.0) << (b1 & 31);
      }
    }
  } else {
    if (tid < N) sw[0] = (uint32_t)(p.d[2 * tid] < 0.0) | ((uint32_t)(p.d[2 * tid + 1] < 0.0) << 1);
  }

  // The bins this thread evaluates in the pruned pass (slot b: Z_{k_b} for
  // b < l, Z_{N - k_{b-l}} for l <= b < 2l).
  int bin[BPT];
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    const int b = tid + u * THREADS;
    bin[u] = -1;
    if (b < 2 * l) {
      const int t = b < l ? b : b - l;
      const int q = p.R[t];
      const int k = q <= N ? q : 2 * N - q;
      bin[u] = (b < l ? k : N - k) & (N - 1);
    }
  }
  // The column this thread assembles: post-twiddle e^{-2 pi i k / n} and scale.
  int kind = 0;
  V pw = make2<V>((T)1, (T)0);
  T scale = (T)0;
  if (tid < l) {
    const int q = p.R[tid];
    const int k = q <= N ? q : 2 * N - q;
    kind = q > N ? 2 : ((q == 0 || q == N) ? 0 : 1);
    double sv, cv;
    sincospi((double)k / (double)N, &sv, &cv);
    pw = make2<V>((T)cv, (T)(-sv));
    scale = (T)(kind == 0 ? 1.0 / sqrt((double)l) : sqrt(2.0 / (double)l));
  }
  __syncthreads();

  const int voff = tid * (int)sizeof(V);
  V v[P >= 1 ? E : 1];
  auto load_row = [&](int64_t row) __attribute__((always_inline)) {
    const __amdgpu_buffer_rsrc_t rs = row_rsrc(static_cast<const T*>(p.A) + row * p.lda, 2 * (int64_t)N);
    if constexpr (P >= 1) {
      if (tid < NB) {
#pragma unroll
        for (int r = 0; r < E; ++r) v[r] = load_pair<VEC>(rs, voff, r * NB * (int)sizeof(V), (V*)nullptr);
      }
    } else {
      if (tid < N) v[0] = load_pair<VEC>(rs, voff, 0, (V*)nullptr);
    }
  };

  T* __restrict__ Y = static_cast<T*>(p.Y);
  int64_t row = blockIdx.x;
  if (row < p.m) load_row(row);
  for (; row < p.m; row += gridDim.x) {
    if constexpr (P >= 1) {
      if (tid < NB) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
          v[r].x = flip_if(v[r].x, sw[(2 * r) >> 5], (2 * r) & 31);
          v[r].y = flip_if(v[r].y, sw[(2 * r + 1) >> 5], (2 * r + 1) & 31);
        }
        RegDFT<E>::run(v);
      }
      __syncthreads();  // the previous row's pruned pass has read `data`
      if (tid < NB) {
        V* w0 = data + tid * (E + 1);
#pragma unroll
        for (int r = 0; r < E; ++r) w0[r] = v[r];
      }
      __syncthreads();
    } else {
      __syncthreads();
      if (tid < N) {
        V z = v[0];
        z.x = flip_if(z.x, sw[0], 0);
        z.y = flip_if(z.y, sw[0], 1);
        data[tid] = z;
      }
      __syncthreads();
    }
    // The next row streams in while this one is transformed.
    if (row + gridDim.x < p.m) load_row(row + gridDim.x);

#pragma unroll
    for (int pass = 1; pass < P; ++pass) {
      const int Ns = 1 << (pass * LOGE);
      const int L = Ns * E;
      const int k = tid & (Ns - 1);
      V u[E];
      if (tid < NB) {
        const V* r0 = data + tid + (tid >> LOGE);
#pragma unroll
        for (int r = 0; r < E; ++r) u[r] = r0[r * (NB + NB / E)];
        // twiddle w_L^{r k}; with at most two full passes L = E^2 and k < E
        const V* tk = twp + k;
#pragma unroll
        for (int r = 1; r < E; ++r) u[r] = cmul(u[r], tk[r * E]);
        RegDFT<E>::run(u);
      }
      __syncthreads();
      if (tid < NB) {
        const int g = tid >> (pass * LOGE);
        V* w0 = data + g * (L + L / E) + k + (k >> LOGE);
#pragma unroll
        for (int r = 0; r < E; ++r) w0[r * (Ns + Ns / E)] = u[r];
      }
      __syncthreads();
    }

    // Pruned last pass: Z_b = sum_r data[j + r NSF] w_N^{r b}, j = b mod NSF.
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
      const int b = bin[u];
      if (b >= 0) {
        const int j = b & (NSF - 1);
        const V* f0 = data + j + (j >> LOGE);
        V w[F];
        unit_powers<F>(w, cmul(thi[b >> G::LOGLO], tlo[b & (G::NLO - 1)]));
        V acc = f0[0];
#pragma unroll
        for (int r = 1; r < F; ++r) acc += cmul(f0[r * (NSF + NSF / E)], w[r]);
        zbuf[tid + u * THREADS] = acc;
      }
    }
    __syncthreads();
    if (tid < l) {
      const V z1 = zbuf[tid];
      const V z2 = zbuf[l + tid];
      const T half = (T)0.5;
      const V ek = make2<V>((z1.x + z2.x) * half, (z1.y - z2.y) * half);
      const V ok = make2<V>((z1.y + z2.y) * half, (z2.x - z1.x) * half);
      const V x = ek + cmul(pw, ok);
      Y[row * l + tid] = kind == 2 ? -scale * x.y : scale * x.x;
    }
  }
}

template <typename T, int LOGN>
hipError_t launch_rows(const SrftRowParams& p, hipStream_t st) {
  typedef SrftGeom<T, LOGN> G;
  // Workgroups per CU allowed by LDS (160 KB per CU on gfx950), at most 8.
  const int per_cu = (int)std::min<size_t>(8, std::max<size_t>(1, (160 * 1024) / G::LDS));
  const int64_t grid = std::min<int64_t>(p.m, (int64_t)256 * per_cu);
  if (p.vec)
    hipLaunchKernelGGL((srft_rows_kernel<T, LOGN, true>), dim3((unsigned)grid), dim3(G::THREADS), 0, st, p);
  else
    hipLaunchKernelGGL((srft_rows_kernel<T, LOGN, false>), dim3((unsigned)grid), dim3(G::THREADS), 0, st, p);
  return hipGetLastError();
}

template <typename T, int LOGN, int MAXLOG>
hipError_t dispatch_rows(int logn, const SrftRowParams& p, hipStream_t st) {
  if (logn == LOGN) return launch_rows<T, LOGN>(p, st);
  if constexpr (LOGN < MAXLOG) return dispatch_rows<T, LOGN + 1, MAXLOG>(logn, p, st);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_srft_rows(int dtype, const void* A, int64_t lda, int64_t m, int64_t n, int32_t l,
                            const double* d, const int32_t* R, void* Y, hipStream_t st) {
  SrftRowParams p{};
  p.A = A;
  p.lda = lda;
  p.m = m;
  p.l = l;
  p.d = d;
  p.R = R;
  p.Y = Y;
  const size_t es = dtype == RSVD_F64 ? 8 : 4;
  p.vec = (lda % 2 == 0 && (reinterpret_cast<uintptr_t>(A) % (2 * es)) == 0) ? 1 : 0;
  int logn = 0;
  while ((int64_t{1} << (logn + 1)) < n) ++logn;  // n = 2^(logn+1)
  if ((int64_t{2} << logn) != n || logn < 2) return hipErrorInvalidValue;
  if (dtype == RSVD_F64) {
    if (logn > SRFT_MAX_LOGN_F64) return hipErrorInvalidValue;
    return dispatch_rows<double, 2, SRFT_MAX_LOGN_F64>(logn, p, st);
  }
  if (logn > SRFT_MAX_LOGN_F32) return hipErrorInvalidValue;
  return dispatch_rows<float, 2, SRFT_MAX_LOGN_F32>(logn, p, st);
}

}  // namespace rsvd
