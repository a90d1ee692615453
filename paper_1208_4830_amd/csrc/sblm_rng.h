// sblm_rng.h -- Philox4x64-10 counter-based generator (Salmon, Moraes, Dror
// & Shaw 2011) and the maps of its 64-bit words to the unit interval and to
// small integers, shared by the device code of the library.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace sblm {

// ---------------------------------------------------------------- Philox

struct u64x4 {
  uint64_t v[4];
};

__device__ __forceinline__ u64x4 philox4x64_10(uint64_t c0, uint64_t c1,
                                               uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  // round multipliers and Weyl key increments of Philox4x64
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return {{c0, c1, c2, c3}};
}

struct Stream {
  uint64_t seed, lc, gen;
  __device__ __forceinline__ uint64_t draw(uint64_t purpose, uint64_t row,
                                           uint64_t j) const {
    const u64x4 b = philox4x64_10(gen, purpose, row, j >> 2, seed, lc);
    return b.v[j & 3];
  }
};

__device__ __forceinline__ double u01(uint64_t x) {
  return ((double)(x >> 12) + 0.5) * 0x1p-52;
}
__device__ __forceinline__ uint32_t below(uint64_t x, uint32_t n) {
  return (uint32_t)(((x >> 32) * (uint64_t)n) >> 32);
}

}  // namespace sblm
