// Stage B for symmetric and positive semidefinite A (Algorithms 5.3 and 5.5):
// the two small kernels around the shared ones (the products with A, the short
// products, the Gram, the Cholesky factorization and the eigensolver).
//
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
  for (int idx = threadIdx.x; idx < l * l; idx += 256) {
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
  const int tid = threadIdx.x, l = p.l, k = p.k;
  if (tid == 0) {
    if (p.by_magnitude) {
      int i = 0, j = l - 1;
      for (int c = 0; c < k; ++c) {
        const double a = p.lam[i], b = p.lam[j];
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
  for (int c = tid; c < k; c += 256) {
    const double v = p.by_magnitude ? p.lam[perm[c]] : p.sig[c] * p.sig[c];
    if (p.dtype == RSVD_F64) ((double*)p.Lam)[c] = v;
    else ((float*)p.Lam)[c] = (float)v;
  }
  if (p.XU) {
    for (int idx = tid; idx < l * k; idx += 256) {
      const int r = idx / k, c = idx - r * k;
      const double v = p.Uh[(int64_t)r * l + perm[c]];
      if (p.dtype == RSVD_F64) ((double*)p.XU)[idx] = v;
      else ((float*)p.XU)[idx] = (float)v;
    }
  }
}

}  // namespace

hipError_t launch_sym_gram(const SymGramParams& p, hipStream_t st) {
  if (p.l < 1 || p.l > RSVD_MAX_L || p.ldb < p.l || p.Lg < p.l || !p.B || !p.G) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sym_gram_kernel, dim3(1), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_eig_pick(const EigPickParams& p, hipStream_t st) {
  if (p.l < 1 || p.l > RSVD_MAX_L || p.k < 1 || p.k > p.l || !p.lam || !p.Lam) return hipErrorInvalidValue;
  if ((p.XU && !p.Uh) || (!p.by_magnitude && !p.sig)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(eig_pick_kernel, dim3(1), dim3(256), 0, st, p);
  return hipGetLastError();
}

}  // namespace rsvd
