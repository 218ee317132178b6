// Random test matrices of Stage A, drawn on the device.
//
// Gaussian Omega (Algorithm 4.1, step 1): one thread per quad of four
// horizontally adjacent entries, one Philox4x64-10 call per quad, Box-Muller
// on the two uniform pairs.  Entries are formed in FP64 and rounded once to
// the element type.
//
// SRFT (Section 4.6): the diagonal D of random +-1 signs (one thread per
// coordinate) and the sampler R of l coordinates drawn without replacement by
// a partial Fisher-Yates shuffle of [0, n).  Step t swaps positions t and
// j_t >= t and emits the value then at position t.  The draws j_t are
// independent, so the shuffle is resolved in parallel: the value at position
// x just before step t is x itself unless an earlier step s < t swapped into
// x (j_s = x); then it is the value that sat at position s just before step s.
// Each thread follows that chain back for its own t (time strictly decreases,
// so the walk ends) and needs no permutation array.
#include "common.hpp"
#include "philox.hpp"

namespace rsvd {

namespace {

constexpr double kTwoPi = 0x1.921fb54442d18p+2;  // the double nearest 2*pi

template <typename T>
__device__ __forceinline__ void omega_body(const OmegaParams& p, const int bid) {
  const int32_t l = p.l;
  const int32_t qpr = (l + 3) / 4;
  const int64_t t = (int64_t)bid * 256 + threadIdx.x;
  if (t >= p.n * qpr) return;
  const int64_t i = t / qpr;
  const int32_t j0 = (int32_t)(t - i * qpr) * 4;
  const Philox4 w = philox4x64_10((uint64_t)t, p.sid, 0ull, 0ull, p.seed, 0ull);
  const double u0 = philox_uniform(w.w[0]), u1 = philox_uniform(w.w[1]);
  const double u2 = philox_uniform(w.w[2]), u3 = philox_uniform(w.w[3]);
  const double r01 = sqrt(-2.0 * log(u0));
  const double r23 = sqrt(-2.0 * log(u2));
  const double th01 = kTwoPi * u1;
  const double th23 = kTwoPi * u3;
  double g[4];
  g[0] = r01 * cos(th01);
  g[1] = r01 * sin(th01);
  g[2] = r23 * cos(th23);
  g[3] = r23 * sin(th23);
  T* row = static_cast<T*>(p.omega) + i * l;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (j0 + r < l) row[j0 + r] = (T)g[r];
}

template <typename T>
__global__ __launch_bounds__(256) void omega_kernel(const OmegaParams p) { omega_body<T>(p, blockIdx.x); }

template <typename T>
__global__ __launch_bounds__(256) void omega_batched(const OmegaParams* __restrict__ ps, const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  omega_body<T>(ps[b.item], b.local);
}

__global__ __launch_bounds__(256) void srft_signs_kernel(double* __restrict__ d, int64_t n, uint64_t seed,
                                                         uint64_t sid) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const Philox4 w = philox4x64_10((uint64_t)p, sid, 1ull, 0ull, seed, 0ull);
  d[p] = 1.0 - 2.0 * (double)(w.w[0] & 1ull);
}

// One workgroup; l <= RSVD_MAX_L.
__global__ __launch_bounds__(256) void srft_sample_kernel(int32_t* __restrict__ R, int64_t n, int32_t l,
                                                          uint64_t seed, uint64_t sid) {
  __shared__ int32_t J[RSVD_MAX_L];
  for (int32_t t = threadIdx.x; t < l; t += blockDim.x) {
    const Philox4 w = philox4x64_10((uint64_t)t, sid, 2ull, 0ull, seed, 0ull);
    const double u = philox_uniform(w.w[0]);
    int64_t j = (int64_t)t + (int64_t)floor(u * (double)(n - t));
    if (j > n - 1) j = n - 1;
    J[t] = (int32_t)j;
  }
  __syncthreads();
  for (int32_t t = threadIdx.x; t < l; t += blockDim.x) {
    int32_t x = J[t];
    int32_t time = t;
    for (;;) {
      int32_t last = -1;
      for (int32_t s = time - 1; s >= 0; --s) {
        if (J[s] == x) {
          last = s;
          break;
        }
      }
      if (last < 0) break;
      x = last;
      time = last;
    }
    R[t] = x;
  }
}

}  // namespace

int64_t omega_blocks(const OmegaParams& p) { return (p.n * ((p.l + 3) / 4) + 255) / 256; }

hipError_t launch_omega(int dtype, void* omega, int64_t n, int32_t l, uint64_t seed, uint64_t sid,
                        hipStream_t st) {
  const OmegaParams p{omega, n, l, seed, sid};
  const dim3 grid((unsigned)omega_blocks(p));
  if (dtype == RSVD_F64)
    hipLaunchKernelGGL(omega_kernel<double>, grid, dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(omega_kernel<float>, grid, dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_omega_batched(int dtype, const OmegaParams* ps, const BlockMap* bm, int64_t nblocks,
                                hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (dtype == RSVD_F64)
    hipLaunchKernelGGL(omega_batched<double>, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
  else
    hipLaunchKernelGGL(omega_batched<float>, dim3((unsigned)nblocks), dim3(256), 0, st, ps, bm);
  return hipGetLastError();
}

hipError_t launch_srft_draw(double* d, int32_t* R, int64_t n, int32_t l, uint64_t seed, uint64_t sid,
                            hipStream_t st) {
  if (l < 1 || l > RSVD_MAX_L || l > n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(srft_signs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, n, seed, sid);
  hipLaunchKernelGGL(srft_sample_kernel, dim3(1), dim3(128), 0, st, R, n, l, seed, sid);
  return hipGetLastError();
}

}  // namespace rsvd
