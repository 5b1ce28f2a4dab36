// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), device side.
//
// One block maps a 128-bit counter and a 64-bit key to 128 random bits by ten
// rounds; each round multiplies two counter words by fixed odd constants
// (32x32 -> 64 bits), swaps the halves into place and mixes in the key, and
// the key advances by a Weyl increment between rounds.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amdalias {

struct u32x4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32 x 32 -> 64-bit product per word (a single multiply-add
    // instruction gives both halves)
    const uint64_t p0 = (uint64_t)M0 * c.x, p1 = (uint64_t)M1 * c.z;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    u32x4 n;
    n.x = hi1 ^ c.y ^ k0;
    n.y = lo1;
    n.z = hi0 ^ c.w ^ k1;
    n.w = lo0;
    c = n;
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// floor(x * r / 2^64) for a 64-bit x and a 32-bit r, exactly (the value of
// the 64 x 64 multiply-high when r < 2^32): with x = xh 2^32 + xl,
// x r / 2^64 = (xh r + xl r / 2^32) / 2^32, and dropping the fraction of
// xl r / 2^32 does not change the floor; xh r + (xl r >> 32) < 2^64.
__device__ __forceinline__ uint64_t mulhi_u64_u32(uint64_t x, uint32_t r) {
  const uint64_t lo = (uint64_t)(uint32_t)x * r;
  const uint64_t hi = (x >> 32) * (uint64_t)r;
  return (hi + (lo >> 32)) >> 32;
}

}  // namespace amdalias
