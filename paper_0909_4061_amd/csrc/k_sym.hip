// Stage B for symmetric and positive semidefinite A (Algorithms 5.3 and 5.5)
// and the single-pass Algorithm 5.6: the small kernels around the shared ones
// (the products with A, the short products, the Gram, the Cholesky
// factorization and the eigensolver).
//
//   cross    : C = X1^T X2 for tall X1 (rows x c1) and X2 (rows x c2), a long
//              contraction into a small output: exact FP64 partial products per
//              chunk of rows, then a fixed-order sum, written in the element
//              type or, for c1 == c2, as the symmetric part into the FP64 Gram
//              layout (B = Q^T (A Q) of Algorithms 5.3 / 5.5).
//   sym_gram : G (FP64, upper triangle, row stride Lg) = (B + B^T) / 2 for an
//              l x l matrix B in the element type (B = Q^T A Q is symmetric in
//              exact arithmetic only).
//   eig_pick : the kept eigenpairs of the l x l eigendecomposition, whose
//              eigenvalues arrive in decreasing order of value.  Magnitude
//              order (Algorithm 5.3, symmetric A of either sign): the k of
//              largest |lambda| are a merge of the two ends of that list
//              (equal magnitudes: the positive one first); lambda and the
//              matching eigenvector columns are written in the element type.
//              Value order (Algorithm 5.5): lambda_j = sig_j^2 for j < k.
#include "common.hpp"

namespace rsvd {

namespace {

template <typename T>
__device__ __forceinline__ double ld_elem(const void* p, int64_t i) {
  return (double)reinterpret_cast<const T*>(p)[i];
}

__global__ __launch_bounds__(256) void sym_gram_kernel(const SymGramParams p) {
  const int l = p.l;
  for (int idx = blockIdx.x * 256 + threadIdx.x; idx < l * l; idx += 256 * gridDim.x) {
    const int i = idx / l, j = idx - i * l;
    if (i > j) continue;
    double a, b;
    if (p.dtype == RSVD_F64) {
      a = ld_elem<double>(p.B, (int64_t)i * p.ldb + j);
      b = ld_elem<double>(p.B, (int64_t)j * p.ldb + i);
    } else {
      a = ld_elem<float>(p.B, (int64_t)i * p.ldb + j);
      b = ld_elem<float>(p.B, (int64_t)j * p.ldb + i);
    }
    p.G[(int64_t)i * p.Lg + j] = 0.5 * (a + b);
  }
}

__global__ __launch_bounds__(256) void eig_pick_kernel(const EigPickParams p) {
  __shared__ int perm[RSVD_MAX_L];
  __shared__ double lam[RSVD_MAX_L];
  const int tid = threadIdx.x, l = p.l, k = p.k;
  for (int i = tid; i < l; i += 256) lam[i] = p.lam[i];
  __syncthreads();
  if (tid == 0) {
    if (p.by_magnitude) {
      int i = 0, j = l - 1;
      for (int c = 0; c < k; ++c) {
        const double a = lam[i], b = lam[j];
        const bool front = fabs(a) > fabs(b) || (fabs(a) == fabs(b) && a >= b);
        perm[c] = front ? i : j;
        if (front) ++i;
        else --j;
      }
    } else {
      for (int c = 0; c < k; ++c) perm[c] = c;
    }
  }
  __syncthreads();
  for (int c = tid; blockIdx.x == 0 && c < k; c += 256) {
    const double v = p.by_magnitude ? lam[perm[c]] : p.sig[c] * p.sig[c];
    if (p.dtype == RSVD_F64) ((double*)p.Lam)[c] = v;
    else ((float*)p.Lam)[c] = (float)v;
  }
  if (p.XU) {
    for (int idx = blockIdx.x * 256 + tid; idx < l * k; idx += 256 * gridDim.x) {
      const int r = idx / k, c = idx - r * k;
      const double v = p.Uh[(int64_t)r * l + perm[c]];
      if (p.dtype == RSVD_F64) ((double*)p.XU)[idx] = v;
      else ((float*)p.XU)[idx] = (float)v;
    }
  }
}

// Partial cross products of one chunk of CROSS_ROWS rows: part[b] (Lg x Lg,
// FP64) = X1_b^T X2_b (c1 x c2), X1 and X2 rows x c1 / rows x c2 in the element
// type.  FP32 entries are exact in FP64, so the products are exact; the chunk's
// rows are staged in LDS and each thread accumulates an 8 x 8 block of the
// output in registers.
template <typename T>
__global__ __launch_bounds__(256) void cross_partial_kernel(const CrossParams p) {
  constexpr int R = CROSS_ROWS;
  __shared__ __attribute__((aligned(16))) T s1[R][RSVD_MAX_L];  // the chunk in the element type (2 per CU for FP32)
  __shared__ __attribute__((aligned(16))) T s2[R][RSVD_MAX_L];
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  const int64_t r0 = (int64_t)blockIdx.x * R;
  const int nr = (int)min<int64_t>(R, p.rows - r0);
  const T* __restrict__ x1 = (const T*)p.X1;
  const T* __restrict__ x2 = (const T*)p.X2;
  // every load of the stage issued before the first store (fixed count per thread)
  constexpr int PER = R * RSVD_MAX_L / 256;
  T t1[PER], t2[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    // branch-free: clamped addresses, the values outside the block selected to zero afterwards
    const int idx = tid + 256 * q, r = idx / RSVD_MAX_L, c = idx - r * RSVD_MAX_L;
    const int64_t rr = r0 + min(r, nr - 1);
    const T a = x1[rr * p.ld1 + min(c, p.c1 - 1)];
    const T b = x2[rr * p.ld2 + min(c, p.c2 - 1)];
    t1[q] = (r < nr && c < p.c1) ? a : T(0);
    t2[q] = (r < nr && c < p.c2) ? b : T(0);
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + 256 * q, r = idx / RSVD_MAX_L, c = idx - r * RSVD_MAX_L;
    s1[r][c] = t1[q];
    s2[r][c] = t2[q];
  }
  __syncthreads();
  double acc[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[a][b] = 0.0;
  if (8 * ti < p.c1 && 8 * tj < p.c2) {
    // rows past the matrix were staged as zeros: a fixed trip count the compiler pipelines
#pragma unroll 4
    for (int r = 0; r < R; ++r) {
      double u[8], v[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        u[a] = (double)s1[r][8 * ti + a];
        v[a] = (double)s2[r][8 * tj + a];
      }
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = fma(u[a], v[b], acc[a][b]);
    }
  }
  double* __restrict__ part = p.part + (int64_t)blockIdx.x * p.Lg * p.Lg;
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int i = 8 * ti + a, j = 8 * tj + b;
      if (i < p.c1 && j < p.c2) part[(int64_t)i * p.Lg + j] = acc[a][b];
    }
}

// Sum of the nblk partial cross products in chunk order.  sym == 0: out
// (c1 x c2, element type, row stride ldo) = the sum.  sym == 1 (c1 == c2):
// G (FP64 upper triangle, stride Lg) = its symmetric part (C + C^T) / 2.
// Each workgroup takes 64 outputs; its four waves sum every fourth partial (eight
// loads in flight each) and the four sums are added in a fixed order.
__global__ __launch_bounds__(256) void cross_reduce_kernel(const CrossParams p) {
  __shared__ double red[2][4][64];
  const int tid = threadIdx.x, q4 = tid >> 6, t = tid & 63;
  const int64_t e = (int64_t)blockIdx.x * 64 + t;
  const bool live = e < (int64_t)p.c1 * p.c2;
  const int i = live ? (int)(e / p.c2) : 0, j = live ? (int)(e - (int64_t)i * p.c2) : 0;
  const bool want = live && !(p.sym && i > j);
  const int64_t LL = (int64_t)p.Lg * p.Lg;
  double a = 0.0, b = 0.0;
  if (want) {
#pragma unroll 8
    for (int64_t q = q4; q < p.nblk; q += 4) {
      a += p.part[q * LL + (int64_t)i * p.Lg + j];
      if (p.sym) b += p.part[q * LL + (int64_t)j * p.Lg + i];
    }
  }
  red[0][q4][t] = a;
  red[1][q4][t] = b;
  __syncthreads();
  if (q4 != 0 || !want) return;
  a = (red[0][0][t] + red[0][1][t]) + (red[0][2][t] + red[0][3][t]);
  b = (red[1][0][t] + red[1][1][t]) + (red[1][2][t] + red[1][3][t]);
  if (p.sym) {
    p.G[(int64_t)i * p.Lg + j] = 0.5 * (a + b);
  } else if (p.dtype == RSVD_F64 || p.out_f64) {
    ((double*)p.out)[(int64_t)i * p.ldo + j] = a;
  } else {
    ((float*)p.out)[(int64_t)i * p.ldo + j] = (float)a;
  }
}

__global__ __launch_bounds__(256) void sylv_div_kernel(double* X, int64_t ld, const double* d2, const double* d1,
                                                       int l) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= l * l) return;
  const int i = e / l, j = e - i * l;
  X[(int64_t)i * ld + j] /= d2[i] + d1[j];
}

}  // namespace

hipError_t launch_sylv_div(double* X, int64_t ld, const double* d2, const double* d1, int32_t l, hipStream_t st) {
  if (l < 1 || l > RSVD_MAX_L || ld < l || !X || !d2 || !d1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sylv_div_kernel, dim3((unsigned)((l * l + 255) / 256)), dim3(256), 0, st, X, ld, d2, d1, l);
  return hipGetLastError();
}

int64_t cross_blocks(int64_t rows) { return (rows + CROSS_ROWS - 1) / CROSS_ROWS; }

hipError_t launch_cross(const CrossParams& p, hipStream_t st) {
  if (p.rows < 1 || p.c1 < 1 || p.c2 < 1 || p.c1 > RSVD_MAX_L || p.c2 > RSVD_MAX_L || p.Lg < p.c1 ||
      p.Lg < p.c2 || p.ld1 < p.c1 || p.ld2 < p.c2 || p.nblk != cross_blocks(p.rows) || !p.X1 || !p.X2 || !p.part)
    return hipErrorInvalidValue;
  if (p.sym ? (p.c1 != p.c2 || !p.G) : (!p.out || p.ldo < p.c2)) return hipErrorInvalidValue;
  if (p.dtype == RSVD_F64)
    hipLaunchKernelGGL(cross_partial_kernel<double>, dim3((unsigned)p.nblk), dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(cross_partial_kernel<float>, dim3((unsigned)p.nblk), dim3(256), 0, st, p);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t outs = (int64_t)p.c1 * p.c2;
  hipLaunchKernelGGL(cross_reduce_kernel, dim3((unsigned)((outs + 63) / 64)), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_sym_gram(const SymGramParams& p, hipStream_t st) {
  if (p.l < 1 || p.l > RSVD_MAX_L || p.ldb < p.l || p.Lg < p.l || !p.B || !p.G) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sym_gram_kernel, dim3((unsigned)((p.l * p.l + 255) / 256)), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_eig_pick(const EigPickParams& p, hipStream_t st) {
  if (p.l < 1 || p.l > RSVD_MAX_L || p.k < 1 || p.k > p.l || !p.lam || !p.Lam) return hipErrorInvalidValue;
  if ((p.XU && !p.Uh) || (!p.by_magnitude && !p.sig)) return hipErrorInvalidValue;
  // every workgroup merges the (at most 128) eigenvalues itself and gathers its share of the columns
  const int blocks = p.XU ? (p.l * p.k + 255) / 256 : 1;
  hipLaunchKernelGGL(eig_pick_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p);
  return hipGetLastError();
}

}  // namespace rsvd
