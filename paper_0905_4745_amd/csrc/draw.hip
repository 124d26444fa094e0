// Step 1's random quantities drawn by the library (Section 3): the N phases
// of D (uniform on the unit circle; random signs for real data) and the l
// rows of the subsampling S, distinct and in increasing order (sampled
// without replacement, as the paper's experiments do).  Every number comes
// from Philox4x32-10 (rng.hpp) at a counter fixed by (index, draw, stream,
// system), so a draw is reproducible from its seed anywhere:
//   phases   d_j = exp(2 pi i u_j), u_j the 53-bit uniform of the words at
//            (j, draw, 0, sys); real data: d_j = +1 or -1 by the low bit of
//            the third word;
//   indices  Floyd's sampling of l of N: for s < l, t = N - l + s, the words
//            at (s, draw, 1, sys) give r = floor(x (t + 1) / 2^64) with
//            x = word0 2^32 + word1 (uniform in [0, t]); the set gains r,
//            or t when r is already in it.  idx is the set in increasing
//            order.
// The phases are computed on the device (one thread per entry), the indices
// on the host (a sequential choice; O(N) with a bitmap, no sort).
#include "common.hpp"
#include "kernels.hpp"
#include "rng.hpp"

#include <vector>

namespace mn {

// phase j of system sys
template <bool CPLX>
__device__ __forceinline__ void phase_at(uint64_t seed, int64_t j, uint32_t draw, uint32_t sys, void* __restrict__ d) {
  const U32x4 w = srft_words(seed, (uint32_t)j, draw, 0u, sys);
  if constexpr (CPLX) {
    double s, c;
    sincospi(2.0 * unit53(w), &s, &c);
    reinterpret_cast<cd*>(d)[j] = cd{c, s};
  } else {
    reinterpret_cast<double*>(d)[j] = (w.v[2] & 1u) ? -1.0 : 1.0;
  }
}

template <bool CPLX>
__global__ void __launch_bounds__(256) k_draw_phases(uint64_t seed, uint32_t draw, uint32_t sys, int64_t N,
                                                     void* __restrict__ d) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < N) phase_at<CPLX>(seed, j, draw, sys, d);
}

// the phases of systems sys0 .. sys0 + count - 1 in one launch: grid
// (ceil(max N / 256), count), sys = sys0 + blockIdx.y; tab[2 sys] = N of the
// system, tab[2 sys + 1] = byte offset of its phases from d
template <bool CPLX>
__global__ void __launch_bounds__(256) k_draw_phases_batch(uint64_t seed, uint32_t draw, uint32_t sys0,
                                                           const int64_t* __restrict__ tab, char* __restrict__ d) {
  const uint32_t sys = sys0 + blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < tab[2 * sys]) phase_at<CPLX>(seed, j, draw, sys, d + tab[2 * sys + 1]);
}

hipError_t launch_draw_phases(bool cplx, uint64_t seed, int draw, int sys, int64_t N, void* d, hipStream_t st) {
  const dim3 grid((unsigned)ceil_div(N, 256));
  if (cplx)
    hipLaunchKernelGGL((k_draw_phases<true>), grid, dim3(256), 0, st, seed, (uint32_t)draw, (uint32_t)sys, N, d);
  else
    hipLaunchKernelGGL((k_draw_phases<false>), grid, dim3(256), 0, st, seed, (uint32_t)draw, (uint32_t)sys, N, d);
  return hipGetLastError();
}

hipError_t launch_draw_phases_batch(bool cplx, uint64_t seed, int draw, int sys0, int count, int64_t max_n,
                                    const int64_t* tab, void* d, hipStream_t st) {
  if (sys0 < 0 || count < 1 || count > 65535 || max_n < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)ceil_div(max_n, 256), (unsigned)count);
  if (cplx)
    hipLaunchKernelGGL((k_draw_phases_batch<true>), grid, dim3(256), 0, st, seed, (uint32_t)draw, (uint32_t)sys0,
                       tab, reinterpret_cast<char*>(d));
  else
    hipLaunchKernelGGL((k_draw_phases_batch<false>), grid, dim3(256), 0, st, seed, (uint32_t)draw, (uint32_t)sys0,
                       tab, reinterpret_cast<char*>(d));
  return hipGetLastError();
}

void draw_indices(uint64_t seed, int draw, int sys, int64_t N, int64_t l, int32_t* idx) {
  std::vector<uint8_t> chosen((size_t)N, 0);
  for (int64_t s = 0; s < l; ++s) {
    const int64_t t = N - l + s;
    const U32x4 w = srft_words(seed, (uint32_t)s, (uint32_t)draw, 1u, (uint32_t)sys);
    const uint64_t x = ((uint64_t)w.v[0] << 32) | (uint64_t)w.v[1];
    const uint64_t r = (uint64_t)(((unsigned __int128)x * (unsigned __int128)(uint64_t)(t + 1)) >> 64);
    if (chosen[(size_t)r]) chosen[(size_t)t] = 1;
    else chosen[(size_t)r] = 1;
  }
  int64_t k = 0;
  for (int64_t j = 0; j < N; ++j)
    if (chosen[(size_t)j]) idx[k++] = (int32_t)j;
}

}  // namespace mn
