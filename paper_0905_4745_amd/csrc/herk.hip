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

typedef double f64x4 __attribute__((ext_vector_type(4)));

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

// ---------------------------------------------------------------------------
// The same product on the FP64 matrix cores (v_mfma_f64_16x16x4f64; operand
// layouts on gfx950: A lane l -> row l%16, K l/16; B lane l -> column l%16,
// K l/16; D lane l -> rows 4v + l/16, column l%16).
//
// Complex data as real products: with S's entries interleaved (re, im) along
// K (k' = 2k + p), A'(i, k') = (Sr, Si)(k, i) is column i of S read as
// doubles, and
//   Re G_ij = sum_k' A'(i, k') A'(j, k'),
//   Im G_ij = sum_k' A'(i, k') B''(k', j),  B''(2k) = Si(k, j), B''(2k+1) = -Sr(k, j),
// so each 16 x 16 complex block takes two real products over 2l (no flop is
// wasted).  Real data: one product over l.
//
// Workgroup: 256 threads (2 x 2 waves), a 64 x 64 tile of G; each wave a
// 32 x 32 block (2 x 2 MFMA tiles, plus their imaginary parts).  K runs in
// panels of 16 entries of S (32 doubles for complex data): the panel's 64 +
// 64 columns are staged through LDS in FP64 (row stride 2 doubles longer than
// the panel), the next panel loading into registers during the products.
// Tiles entirely below the diagonal exit; split K and the partial layout are
// those of k_herk (k_herk_fold adds the partials).
constexpr int MT = 64;   // tile edge
constexpr int MK = 16;   // K panel (entries of S)

template <typename T>
__global__ void __launch_bounds__(256) k_herk_mf(const T* __restrict__ S, int64_t lds, int64_t l, int64_t m,
                                                 typename HerkW<T>::type* __restrict__ out, int64_t ldo, int64_t ks,
                                                 int partial) {
  constexpr bool CP = VT<T>::cplx;
  constexpr int KD = CP ? 2 * MK : MK;  // doubles per column per panel
  constexpr int LS = KD + 2;            // LDS row stride (doubles)
  __shared__ double As[MT * LS];
  __shared__ double Bs[MT * LS];
  const int64_t r0 = (int64_t)blockIdx.x * MT, c0 = (int64_t)blockIdx.y * MT;
  if (r0 > c0 + MT - 1) return;  // below the diagonal
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = (wv & 1) * 32, wc = (wv >> 1) * 32;  // wave's block in the tile
  const int li = lane & 15, lk = lane >> 4;
  const int64_t k_begin = (int64_t)blockIdx.z * ks;
  const int64_t k_end = k_begin + ks < l ? k_begin + ks : l;
  const int nch = k_end > k_begin ? (int)((k_end - k_begin + MK - 1) / MK) : 0;

  // staging: thread t loads 4 consecutive entries of column t / 4 (rows
  // 4 (t % 4) ..) of both panels
  const int sc = tid >> 2, sk = (tid & 3) * 4;
  T pa[4], pb[4];
  auto load = [&](int ch) {
    const int64_t k0 = k_begin + (int64_t)ch * MK + sk;
    const int64_t ra = r0 + sc, cb = c0 + sc;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = k0 + u;
      pa[u] = (k < k_end && ra < m) ? S[k + ra * lds] : T{};
      pb[u] = (k < k_end && cb < m) ? S[k + cb * lds] : T{};
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if constexpr (CP) {
        As[sc * LS + 2 * (sk + u)] = (double)vre(pa[u]);
        As[sc * LS + 2 * (sk + u) + 1] = (double)vim(pa[u]);
        Bs[sc * LS + 2 * (sk + u)] = (double)vre(pb[u]);
        Bs[sc * LS + 2 * (sk + u) + 1] = (double)vim(pb[u]);
      } else {
        As[sc * LS + sk + u] = (double)pa[u];
        Bs[sc * LS + sk + u] = (double)pb[u];
      }
    }
  };

  f64x4 are[2][2], aim[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) are[i][j] = aim[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  if (nch > 0) {
    load(0);
    store();
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    if (ch + 1 < nch) load(ch + 1);
#pragma unroll
    for (int s = 0; s < KD / 4; ++s) {
      const int kk = 4 * s + lk;
      double a[2], b[2], bi[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[(wr + 16 * t + li) * LS + kk];
        b[t] = Bs[(wc + 16 * t + li) * LS + kk];
        if constexpr (CP) {
          const double o = Bs[(wc + 16 * t + li) * LS + (kk ^ 1)];
          bi[t] = (kk & 1) ? -o : o;
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) are[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], are[i][j], 0, 0, 0);
      if constexpr (CP) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            aim[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bi[j], aim[i][j], 0, 0, 0);
      }
    }
    if (ch + 1 < nch) {
      __syncthreads();  // every wave is done with this panel
      store();
    }
    __syncthreads();
  }

  // upper triangle r <= c of G (or of this split's partial)
  using W = typename HerkW<T>::type;
  W* dst = out + (partial ? (int64_t)blockIdx.z * m * ldo : 0);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t c = c0 + wc + 16 * j + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + wr + 16 * i + 4 * v + lk;
        if (r <= c && c < m) {
          if constexpr (CP) dst[r + c * ldo] = cd{are[i][j][v], aim[i][j][v]};
          else dst[r + c * ldo] = are[i][j][v];
        }
      }
    }
}

template <typename T>
hipError_t herk_mf_impl(const void* S, int64_t lds, int64_t l, int64_t m, void* G, int64_t ldg, void* Cp, int splits,
                        int64_t ks, hipStream_t st) {
  using W = typename HerkW<T>::type;
  const dim3 grid((unsigned)ceil_div(m, MT), (unsigned)ceil_div(m, MT), (unsigned)splits);
  if (splits == 1) {
    hipLaunchKernelGGL((k_herk_mf<T>), grid, dim3(256), 0, st, reinterpret_cast<const T*>(S), lds, l, m,
                       reinterpret_cast<W*>(G), ldg, ks, 0);
  } else {
    hipLaunchKernelGGL((k_herk_mf<T>), grid, dim3(256), 0, st, reinterpret_cast<const T*>(S), lds, l, m,
                       reinterpret_cast<W*>(Cp), m, ks, 1);
    hipLaunchKernelGGL((k_herk_fold<W>), dim3((unsigned)ceil_div(m, 256), (unsigned)m), dim3(256), 0, st,
                       reinterpret_cast<const W*>(Cp), splits, m, reinterpret_cast<W*>(G), ldg);
  }
  return hipGetLastError();
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

hipError_t launch_herk_mf(int dtype, const void* S, int64_t lds, int64_t l, int64_t m, void* G, int64_t ldg,
                          void* Cp, int splits, int64_t ks, hipStream_t st) {
  if (m < 1 || l < 1 || lds < l || ldg < m || splits < 1 || ks < 1 || (int64_t)splits * ks < l) return hipErrorInvalidValue;
  if (splits > 1 && Cp == nullptr) return hipErrorInvalidValue;
  if (m > 65535) return hipErrorInvalidValue;
  switch (dtype) {
    case 0: return herk_mf_impl<cd>(S, lds, l, m, G, ldg, Cp, splits, ks, st);
    case 1: return herk_mf_impl<cf>(S, lds, l, m, G, ldg, Cp, splits, ks, st);
    case 2: return herk_mf_impl<double>(S, lds, l, m, G, ldg, Cp, splits, ks, st);
    case 3: return herk_mf_impl<float>(S, lds, l, m, G, ldg, Cp, splits, ks, st);
  }
  return hipErrorInvalidValue;
}

int herk_mf_tile() { return MT; }

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
