// Counter-based random numbers for the SRFT's draws (Section 3: D's phases and
// the subsampled rows of S): Philox4x32-10 as defined by Salmon, Moraes, Dror
// and Shaw ("Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds
// of two 32 x 32 -> 64-bit multiplications on a four-word counter, the
// two-word key advanced by the Weyl constants between rounds.  Usable on the
// host and on the device (same integer arithmetic, same outputs).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mn {

struct U32x4 {
  uint32_t v[4];
};

__host__ __device__ inline U32x4 philox4x32_10(U32x4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;  // round multipliers
  constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;  // key increments
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t p0 = (uint64_t)kM0 * c.v[0];
    const uint64_t p1 = (uint64_t)kM1 * c.v[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = U32x4{{hi1 ^ c.v[1] ^ k0, lo1, hi0 ^ c.v[3] ^ k1, lo0}};
  }
  return c;
}

// The words of one draw: counter (index, draw, stream, system), key = seed.
// Stream 0 gives the phases, stream 1 the subsample choices.
__host__ __device__ inline U32x4 srft_words(uint64_t seed, uint32_t index, uint32_t draw, uint32_t stream,
                                            uint32_t sys) {
  return philox4x32_10(U32x4{{index, draw, stream, sys}}, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// 53-bit uniform in [0, 1) from the first two words
__host__ __device__ inline double unit53(const U32x4& w) {
  return (double)(((uint64_t)(w.v[0] >> 5) << 26) | (uint64_t)(w.v[1] >> 6)) * 0x1.0p-53;
}

}  // namespace mn
