// Achievable-peak probes for the roofline fractions the benchmark reports:
// how fast this GPU streams HBM and issues MFMA work, measured with kernels
// written like the library's own rather than taken from a datasheet.
//
//   hbm_read_kernel : every byte of a buffer read once with 16-byte loads,
//                     eight loads in flight per thread, grid-stride over the
//                     buffer; one value per workgroup written (so the loads
//                     are not dead).
//   mfma_loop_kernel: each wave issues `iters` rounds of four independent MFMA
//                     accumulations (BF16 32x32x16, FP32 32x32x2 or FP64
//                     16x16x4) on register operands, then writes its
//                     accumulators.
#include "common.hpp"

namespace rsvd {

namespace {

constexpr int CEIL_THREADS = 256;
constexpr int CEIL_UNROLL = 8;

typedef float f32x4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(CEIL_THREADS) void hbm_read_kernel(const f32x4v* __restrict__ buf, int64_t nvec,
                                                                float* __restrict__ sink) {
  __shared__ float red[CEIL_THREADS];
  const int64_t stride = (int64_t)gridDim.x * CEIL_THREADS;
  f32x4v acc = {0.f, 0.f, 0.f, 0.f};
  int64_t i = (int64_t)blockIdx.x * CEIL_THREADS + threadIdx.x;
  for (; i + (CEIL_UNROLL - 1) * stride < nvec; i += CEIL_UNROLL * stride) {
    f32x4v v[CEIL_UNROLL];
#pragma unroll
    for (int u = 0; u < CEIL_UNROLL; ++u) v[u] = __builtin_nontemporal_load(buf + i + u * stride);
#pragma unroll
    for (int u = 0; u < CEIL_UNROLL; ++u) acc += v[u];
  }
  for (; i < nvec; i += stride) acc += buf[i];
  red[threadIdx.x] = (acc.x + acc.y) + (acc.z + acc.w);
  __syncthreads();
  for (int s = CEIL_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) sink[blockIdx.x] = red[0];
}

template <int KIND>
__global__ __launch_bounds__(CEIL_THREADS) void mfma_loop_kernel(int64_t iters, float* __restrict__ sink) {
  const int lane = threadIdx.x & 63;
  if (KIND == 0) {  // BF16 32x32x16, FP32 accumulation: 32768 flops per MFMA
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = (__bf16)(0.001f * (float)(lane + e));
      b[e] = (__bf16)(0.002f * (float)(lane - e));
    }
    f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
    for (int64_t it = 0; it < iters; ++it) {
      c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c3, 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int e = 0; e < 16; ++e) s += (c0[e] + c1[e]) + (c2[e] + c3[e]);
    sink[(int64_t)blockIdx.x * CEIL_THREADS + threadIdx.x] = s;
  } else if (KIND == 1) {  // FP32 32x32x2: 4096 flops per MFMA
    const float a = 0.001f * (float)lane, b = 0.002f * (float)(lane + 1);
    f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
    for (int64_t it = 0; it < iters; ++it) {
      c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c3, 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int e = 0; e < 16; ++e) s += (c0[e] + c1[e]) + (c2[e] + c3[e]);
    sink[(int64_t)blockIdx.x * CEIL_THREADS + threadIdx.x] = s;
  } else {  // FP64 16x16x4: 2048 flops per MFMA
    const double a = 0.001 * lane, b = 0.002 * (lane + 1);
    f64x4 c0 = {}, c1 = {}, c2 = {}, c3 = {};
    for (int64_t it = 0; it < iters; ++it) {
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c3, 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) s += (c0[e] + c1[e]) + (c2[e] + c3[e]);
    sink[(int64_t)blockIdx.x * CEIL_THREADS + threadIdx.x] = (float)s;
  }
}

}  // namespace

int64_t ceiling_read_blocks() { return 256 * 8; }

hipError_t launch_hbm_read(const void* buf, size_t bytes, float* sink, hipStream_t st) {
  if (!buf || !sink || bytes < 16 || (reinterpret_cast<uintptr_t>(buf) & 15u) != 0) return hipErrorInvalidValue;
  const int64_t nvec = (int64_t)(bytes / 16);
  hipLaunchKernelGGL(hbm_read_kernel, dim3((unsigned)ceiling_read_blocks()), dim3(CEIL_THREADS), 0, st,
                     reinterpret_cast<const f32x4v*>(buf), nvec, sink);
  return hipGetLastError();
}

hipError_t launch_mfma_loop(int kind, int64_t iters, int64_t blocks, float* sink, hipStream_t st) {
  if (!sink || iters < 1 || blocks < 1 || kind < 0 || kind > 2) return hipErrorInvalidValue;
  const dim3 g((unsigned)blocks);
  if (kind == 0)
    hipLaunchKernelGGL(mfma_loop_kernel<0>, g, dim3(CEIL_THREADS), 0, st, iters, sink);
  else if (kind == 1)
    hipLaunchKernelGGL(mfma_loop_kernel<1>, g, dim3(CEIL_THREADS), 0, st, iters, sink);
  else
    hipLaunchKernelGGL(mfma_loop_kernel<2>, g, dim3(CEIL_THREADS), 0, st, iters, sink);
  return hipGetLastError();
}

}  // namespace rsvd
