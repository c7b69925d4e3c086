// Counter-based random numbers of the library's generators (HIP, gfx950):
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011) and its map of a 32-bit output to (0, 1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppe {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// u = ((x >> 8) + 1/2) 2^-24, strictly inside (0, 1).
__device__ __forceinline__ double unit01(uint32_t x) { return ((double)(x >> 8) + 0.5) * 0x1p-24; }

}  // namespace ppe
