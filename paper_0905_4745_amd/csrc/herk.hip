// Gram matrix G = S* S of the sketch (Step 2 uses only the triangular factor
// of S, and R* R = S* S for the R of any QR of S), FP64, upper triangle, on
// the vector units.  On gfx950 the FP64 fused multiply-add runs at the FP64
// matrix-core rate, so a register-tiled product on the vector units (no
// operand expansion for complex data) is the faster form for large m.
//
// Workgroup: 256 threads, a 128 x 64 tile of G (rows r0 .., columns c0 ..),
// thread t owns rows r0 + t%16 + 16 i (i < 8) and columns c0 + t/16 + 16 j
// (j < 4).  K runs in panels of 16: the panel of S's columns r0 .. r0+127
// and c0 .. c0+63 is staged through LDS in FP64, the next panel loading into
// registers while the current one is used (a panel's products cover the
// latency of the next panel's loads from HBM).  Tiles entirely below the
// diagonal exit at once.  Split K: workgroup z takes rows k of S in
// [z ks, (z+1) ks) and writes its partial tile to Cp (folded by k_herk_fold).
#include "common.hpp"
#include "kernels.hpp"

namespace mn {

namespace {

constexpr int HR = 128;  // tile rows
constexpr int HC = 64;   // tile columns
constexpr int HK = 16;   // K panel

template <typename T> struct HerkW { using type = typename std::conditional<VT<T>::cplx, cd, double>::type; };

// a* b + acc (complex) or a b + acc (real), as fused multiply-adds
__device__ __forceinline__ cd herk_mac(cd a, cd b, cd acc) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
  return acc;
}
__device__ __forceinline__ double herk_mac(double a, double b, double acc) { return fma(a, b, acc); }

template <typename T>
__global__ void __launch_bounds__(256) k_herk(const T* __restrict__ S, int64_t lds, int64_t l, int64_t m,
                                              typename HerkW<T>::type* __restrict__ out, int64_t ldo, int64_t ks,
                                              int partial) {
  using W = typename HerkW<T>::type;
  __shared__ W As[HK][HR + 1];
  __shared__ W Bs[HK][HC + 1];
  const int64_t r0 = (int64_t)blockIdx.x * HR, c0 = (int64_t)blockIdx.y * HC;
  if (r0 > c0 + HC - 1) return;  // below the diagonal
  const int tid = threadIdx.x;
  const int tr = tid & 15, tc = tid >> 4;
  const int64_t k_begin = (int64_t)blockIdx.z * ks;
  const int64_t k_end = k_begin + ks < l ? k_begin + ks : l;
  const int nch = k_end > k_begin ? (int)((k_end - k_begin + HK - 1) / HK) : 0;

  // panel loads: element e = tid + 256 u, k = e % 16, column = e / 16
  // (sixteen consecutive k of one column of S per sixteen lanes)
  constexpr int NA = HR * HK / 256, NB = HC * HK / 256;
  T pa[NA], pb[NB];
  auto load = [&](int ch) {
    const int64_t k0 = k_begin + (int64_t)ch * HK;
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + 256 * u;
      const int64_t k = k0 + (e & (HK - 1)), r = r0 + e / HK;
      pa[u] = (k < k_end && r < m) ? S[k + r * lds] : T{};
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + 256 * u;
      const int64_t k = k0 + (e & (HK - 1)), c = c0 + e / HK;
      pb[u] = (k < k_end && c < m) ? S[k + c * lds] : T{};
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + 256 * u;
      As[e & (HK - 1)][e / HK] = vconv<W>(pa[u]);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + 256 * u;
      Bs[e & (HK - 1)][e / HK] = vconv<W>(pb[u]);
    }
  };

  W acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = vzero<W>();

  if (nch > 0) {
    load(0);
    store();
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    if (ch + 1 < nch) load(ch + 1);
    // one K step's operands live at a time (the 8 x 4 accumulator tile
    // already takes most of the registers)
#pragma unroll 1
    for (int k = 0; k < HK; ++k) {
      W a[8], b[4];
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = As[k][tr + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[k][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = herk_mac(a[i], b[j], acc[i][j]);
    }
    if (ch + 1 < nch) {
      __syncthreads();  // every wave is done with this panel
      store();
    }
    __syncthreads();
  }

  // upper triangle r <= c of G (or of this split's partial)
  W* dst = out + (partial ? (int64_t)blockIdx.z * m * ldo : 0);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t c = c0 + tc + 16 * j;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t r = r0 + tr + 16 * i;
      if (r <= c && c < m) dst[r + c * ldo] = acc[i][j];
    }
  }
}

// G[r + c ldg] = sum of the split partials (upper triangle only).
// grid (ceil(m / 256), m).
template <typename W>
__global__ void __launch_bounds__(256) k_herk_fold(const W* __restrict__ Cp, int splits, int64_t m,
                                                   W* __restrict__ G, int64_t ldg) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= m || r > c) return;
  W s = Cp[r + c * m];
  for (int z = 1; z < splits; ++z) s = vadd(s, Cp[(int64_t)z * m * m + r + c * m]);
  G[r + c * ldg] = s;
}

template <typename T>
hipError_t herk_impl(const void* S, int64_t lds, int64_t l, int64_t m, void* G, int64_t ldg, void* Cp, int splits,
                     int64_t ks, hipStream_t st) {
  using W = typename HerkW<T>::type;
  const dim3 grid((unsigned)ceil_div(m, HR), (unsigned)ceil_div(m, HC), (unsigned)splits);
  if (splits == 1) {
    hipLaunchKernelGGL((k_herk<T>), grid, dim3(256), 0, st, reinterpret_cast<const T*>(S), lds, l, m,
                       reinterpret_cast<W*>(G), ldg, ks, 0);
  } else {
    hipLaunchKernelGGL((k_herk<T>), grid, dim3(256), 0, st, reinterpret_cast<const T*>(S), lds, l, m,
                       reinterpret_cast<W*>(Cp), m, ks, 1);
    hipLaunchKernelGGL((k_herk_fold<W>), dim3((unsigned)ceil_div(m, 256), (unsigned)m), dim3(256), 0, st,
                       reinterpret_cast<const W*>(Cp), splits, m, reinterpret_cast<W*>(G), ldg);
  }
  return hipGetLastError();
}

}  // namespace

int64_t herk_part_elems(int64_t m, int splits) { return splits > 1 ? (int64_t)splits * m * m : 0; }

hipError_t launch_herk(int dtype, const void* S, int64_t lds, int64_t l, int64_t m, void* G, int64_t ldg, void* Cp,
                       int splits, int64_t ks, hipStream_t st) {
  if (m < 1 || l < 1 || lds < l || ldg < m || splits < 1 || ks < 1 || (int64_t)splits * ks < l) return hipErrorInvalidValue;
  if (splits > 1 && Cp == nullptr) return hipErrorInvalidValue;
  if (m > 65535) return hipErrorInvalidValue;  // grid.y of the fold
  switch (dtype) {
    case 0: return herk_impl<cd>(S, lds, l, m, G, ldg, Cp, splits, ks, st);
    case 1: return herk_impl<cf>(S, lds, l, m, G, ldg, Cp, splits, ks, st);
    case 2: return herk_impl<double>(S, lds, l, m, G, ldg, Cp, splits, ks, st);
    case 3: return herk_impl<float>(S, lds, l, m, G, ldg, Cp, splits, ks, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace mn
