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
//     straight from HBM (one 8- or 16-byte load per complex value) with the
//     signs of D applied on the fly;
//   * P passes of a radix-E Stockham FFT (the self-sorting formulation of
//     Govindaraju et al., SC'08): each thread holds one radix-E butterfly in
//     registers, twiddles come from a quarter-wave cosine table in LDS, and
//     the N values live in LDS between passes under an XOR swizzle that keeps
//     the stride-E stores of the first pass free of bank conflicts;
//   * the last radix-F pass is pruned: only the 2l bins Z_k, Z_{N-k} the
//     sampled columns need are evaluated, each as an F-term sum;
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

// exp(-2 pi i idx / N) for 0 <= idx < N from ct[i] = cos(2 pi i / N), 0 <= i <= N/4.
template <typename V, typename T, int LOGN>
__device__ __forceinline__ V root_n(const T* ct, uint32_t idx) {
  constexpr uint32_t Q = (1u << LOGN) / 4;
  const uint32_t qd = idx >> (LOGN - 2);
  const uint32_t rr = idx & (Q - 1);
  const T c0 = ct[rr], s0 = ct[Q - rr];
  T c = (qd & 1) ? -s0 : c0;
  T s = (qd & 1) ? c0 : s0;
  if (qd & 2) {
    c = -c;
    s = -s;
  }
  return make2<V>(c, -s);
}

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
  static constexpr int F = N / NSF;                 // radix of the pruned pass, 2..E
  static constexpr int NB = N / E;                  // butterflies per full pass
  static constexpr int THREADS = NB > 128 ? NB : 128;
  static constexpr size_t LDS = N * 2 * sizeof(T) + (N / 4 + 1) * sizeof(T);
};

template <int LOGE>
__device__ __forceinline__ int swz(int i) {
  return i ^ ((i >> LOGE) & ((1 << LOGE) - 1));
}

template <typename T, int LOGN>
__global__ __launch_bounds__(256) void srft_rows_kernel(SrftRowParams p) {
  typedef typename Vec2<T>::type V;
  typedef SrftGeom<T, LOGN> G;
  constexpr int N = G::N, E = G::E, LOGE = G::LOGE, P = G::P, NSF = G::NSF, F = G::F, NB = G::NB;
  __shared__ V data[N];
  __shared__ T ct[N / 4 + 1];
  const int tid = threadIdx.x;

  for (int i = tid; i <= N / 4; i += blockDim.x) ct[i] = (T)cospi(2.0 * (double)i / (double)N);

  // Signs of D for the 2E real entries this thread loads (bit 2r: real part of
  // its r-th complex value, bit 2r+1: imaginary part).
  uint64_t sbits = 0;
  if constexpr (P >= 1) {
    if (tid < NB) {
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int c = tid + r * NB;
        sbits |= (uint64_t)(p.d[2 * c] < 0.0) << (2 * r);
        sbits |= (uint64_t)(p.d[2 * c + 1] < 0.0) << (2 * r + 1);
      }
    }
  } else {
    if (tid < N) sbits = (uint64_t)(p.d[2 * tid] < 0.0) | ((uint64_t)(p.d[2 * tid + 1] < 0.0) << 1);
  }

  // Sampled column owned by this thread: the bins it needs, the post-twiddle
  // e^{-2 pi i k / n} and the output scale.
  const bool has_col = tid < p.l;
  int zb1 = 0, zb2 = 0, kind = 0;
  V pw = make2<V>((T)1, (T)0);
  T scale = (T)0;
  if (has_col) {
    const int q = p.R[tid];
    int k;
    if (q <= N) {
      k = q;
      kind = (q == 0 || q == N) ? 0 : 1;
    } else {
      k = 2 * N - q;
      kind = 2;
    }
    zb1 = k & (N - 1);
    zb2 = (N - k) & (N - 1);
    double sv, cv;
    sincospi((double)k / (double)N, &sv, &cv);
    pw = make2<V>((T)cv, (T)(-sv));
    scale = (T)(kind == 0 ? 1.0 / sqrt((double)p.l) : sqrt(2.0 / (double)p.l));
  }
  __syncthreads();

  auto eval_bin = [&](int b) __attribute__((always_inline)) {
    const int j = b & (NSF - 1);
    V acc = data[swz<LOGE>(j)];
#pragma unroll
    for (int r = 1; r < F; ++r)
      acc += cmul(data[swz<LOGE>(j + r * NSF)], root_n<V, T, LOGN>(ct, (uint32_t)(r * b) & (N - 1)));
    return acc;
  };

  T* __restrict__ Y = static_cast<T*>(p.Y);
  for (int64_t row = blockIdx.x; row < p.m; row += gridDim.x) {
    const T* __restrict__ a = static_cast<const T*>(p.A) + row * p.lda;
    if constexpr (P >= 1) {
      V v[E];
      if (tid < NB) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const int c = tid + r * NB;
          V z;
          if (p.vec) {
            z = reinterpret_cast<const V*>(a)[c];
          } else {
            z.x = a[2 * c];
            z.y = a[2 * c + 1];
          }
          if ((sbits >> (2 * r)) & 1) z.x = -z.x;
          if ((sbits >> (2 * r + 1)) & 1) z.y = -z.y;
          v[r] = z;
        }
        RegDFT<E>::run(v);
      }
      __syncthreads();  // the previous row's pruned pass has read `data`
      if (tid < NB) {
#pragma unroll
        for (int r = 0; r < E; ++r) data[swz<LOGE>(tid * E + r)] = v[r];
      }
      __syncthreads();
#pragma unroll
      for (int pass = 1; pass < P; ++pass) {
        const int Ns = 1 << (pass * LOGE);
        const int L = Ns * E;
        const int k = tid & (Ns - 1);
        if (tid < NB) {
#pragma unroll
          for (int r = 0; r < E; ++r) v[r] = data[swz<LOGE>(tid + r * NB)];
#pragma unroll
          for (int r = 1; r < E; ++r) v[r] = cmul(v[r], root_n<V, T, LOGN>(ct, (uint32_t)(r * k) * (uint32_t)(N / L)));
          RegDFT<E>::run(v);
        }
        __syncthreads();
        if (tid < NB) {
          const int base = (tid / Ns) * L + k;
#pragma unroll
          for (int r = 0; r < E; ++r) data[swz<LOGE>(base + r * Ns)] = v[r];
        }
        __syncthreads();
      }
    } else {
      __syncthreads();
      if (tid < N) {
        V z;
        z.x = a[2 * tid];
        z.y = a[2 * tid + 1];
        if (sbits & 1) z.x = -z.x;
        if (sbits & 2) z.y = -z.y;
        data[tid] = z;
      }
      __syncthreads();
    }
    if (has_col) {
      const V z1 = eval_bin(zb1);
      const V z2 = eval_bin(zb2);
      const T half = (T)0.5;
      const V ek = make2<V>((z1.x + z2.x) * half, (z1.y - z2.y) * half);
      const V ok = make2<V>((z1.y + z2.y) * half, (z2.x - z1.x) * half);
      const V x = ek + cmul(pw, ok);
      Y[row * p.l + tid] = kind == 2 ? -scale * x.y : scale * x.x;
    }
  }
}

template <typename T, int LOGN>
hipError_t launch_rows(const SrftRowParams& p, hipStream_t st) {
  typedef SrftGeom<T, LOGN> G;
  // Workgroups per CU allowed by LDS (160 KB per CU on gfx950), at most 8.
  const int per_cu = (int)std::min<size_t>(8, std::max<size_t>(1, (160 * 1024) / G::LDS));
  const int64_t grid = std::min<int64_t>(p.m, (int64_t)256 * per_cu);
  hipLaunchKernelGGL((srft_rows_kernel<T, LOGN>), dim3((unsigned)grid), dim3(G::THREADS), 0, st, p);
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
