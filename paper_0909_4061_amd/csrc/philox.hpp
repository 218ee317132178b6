// Device-side Philox4x64-10 and the draws built on it.
//
// Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): each round
// multiplies counter words 0 and 2 by fixed odd constants, keeps the 128-bit
// products' halves, and mixes them with words 1 and 3 and the round key; the
// key is advanced by two Weyl increments between rounds.  The counter is used
// as given, without a pre-increment.
//
// Draw contract (shared with the CPU reference by specification only):
//   key = (seed, 0); uniform u(w) = ((w >> 12) + 1/2) * 2^-52 (exact in FP64);
//   Gaussian quad t of stream s: counter (t, s, 0, 0), Box-Muller on (u0, u1)
//   and (u2, u3) with angle 2*pi*u;
//   SRFT sign p: counter (p, s, 1, 0), d = 1 - 2 (w0 & 1);
//   SRFT sampler step t: counter (t, s, 2, 0), j = min(t + floor(u (n - t)), n - 1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsvd {

struct Philox4 {
  uint64_t w[4];
};

__host__ __device__ inline void philox_round_mul(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
#if defined(__HIP_DEVICE_COMPILE__)
  lo = a * b;
  hi = __umul64hi(a, b);
#else
  unsigned __int128 prod = (unsigned __int128)a * b;
  lo = (uint64_t)prod;
  hi = (uint64_t)(prod >> 64);
#endif
}

__host__ __device__ inline Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                 uint64_t key0, uint64_t key1) {
  const uint64_t kMulA = 0xD2E7470EE14C6C93ull;
  const uint64_t kMulB = 0xCA5A826395121157ull;
  const uint64_t kWeylA = 0x9E3779B97F4A7C15ull;
  const uint64_t kWeylB = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hiA, loA, hiB, loB;
    philox_round_mul(kMulA, c0, hiA, loA);
    philox_round_mul(kMulB, c2, hiB, loB);
    const uint64_t n0 = hiB ^ c1 ^ key0;
    const uint64_t n2 = hiA ^ c3 ^ key1;
    c0 = n0;
    c1 = loB;
    c2 = n2;
    c3 = loA;
    key0 += kWeylA;
    key1 += kWeylB;
  }
  Philox4 out;
  out.w[0] = c0;
  out.w[1] = c1;
  out.w[2] = c2;
  out.w[3] = c3;
  return out;
}

__host__ __device__ inline double philox_uniform(uint64_t w) {
  return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

}  // namespace rsvd
