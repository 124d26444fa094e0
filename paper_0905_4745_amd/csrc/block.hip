// Multi-right-hand-side form of Step 4 (Section 4): k independent CG
// recurrences share every pass over A, so the two products of an iteration
// become block products on the matrix cores.
//
//  * Bulk products W = A* P and Q = A W: split BF16 (x = hi + lo, three
//    products hi*hi + hi*lo + lo*hi, FP32 accumulation) on
//    v_mfma_f32_16x16x32_bf16.  A is converted once per solve into BF16
//    hi/lo planes, row-major for A W and transposed for A* P, so that both
//    products stream their left operand along contiguous rows.
//  * FP64 products (the refinement residual b - A A* y, x = A* y and the
//    triangular preconditioner products X* r, X s): v_mfma_f64_16x16x4f64,
//    reading A or X where they are; that instruction takes one K value per
//    lane, so a transposed operand is read along its stored rows as well.
//
// Complex products run as real ones on the 2 x 2 block form: a complex left
// operand in its interleaved (re, im) layout is a real matrix with twice the
// columns, and a right-hand column c = (br, bi) becomes two real columns,
// (br, -bi) and (bi, br) -- or (br, bi) and (bi, -br) when the left operand is
// conjugated.  The real output columns 2c and 2c + 1 are then Re and Im of
// complex column c.
//
// Operand layouts of the MFMA instructions (measured on gfx950):
//   16x16x32 bf16: A lane l -> row l%16, K 8(l/16)..+7; B lane l -> column
//                  l%16, same K; D lane l -> rows 4(l/16)+v, column l%16.
//   16x16x4 f64:   A lane l -> row l%16, K l/16; B lane l -> column l%16,
//                  K l/16; D lane l -> rows 4v + l/16, column l%16.
// The K order inside one instruction is free as long as both operands use
// the same one; the kernels pick the order that makes each lane's loads
// contiguous.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "batch_dev.hpp"

namespace mn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---- BF16 split ----------------------------------------------------------
__device__ inline uint32_t bf16_bits_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
// x = hi + lo + O(2^-18 |x|); x - hi is exact in FP32
__device__ inline void split2(float x, uint32_t& hi, uint32_t& lo) {
  hi = bf16_bits_rne(x);
  lo = bf16_bits_rne(x - __uint_as_float(hi << 16));
}

template <typename T> struct Elem;
template <> struct Elem<cd> { static constexpr bool cplx = true; };
template <> struct Elem<cf> { static constexpr bool cplx = true; };
template <> struct Elem<double> { static constexpr bool cplx = false; };
template <> struct Elem<float> { static constexpr bool cplx = false; };

// ---------------------------------------------------------------------------
// BF16 hi/lo planes of a row-major M x K matrix (K entries per row; a complex
// entry gives two real columns).  Planes are row-major with ldp >= K' (= K or
// 2K), entries K' .. ldp-1 zero.  Each thread writes 8 values per plane.
template <typename T>
__global__ void __launch_bounds__(256) k_planes(const T* __restrict__ A, int64_t lda, int64_t M, int64_t K,
                                                uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, int64_t ldp) {
  constexpr int E = Elem<T>::cplx ? 2 : 1;
  const int64_t row = blockIdx.y;
  const int64_t k8 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8;
  if (row >= M || k8 >= ldp) return;
  float v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t kk = k8 + q;  // real column
    const int64_t e = kk / E;   // entry
    float x = 0.0f;
    if (e < K) {
      const T a = A[row * lda + e];
      if constexpr (E == 2) x = (kk & 1) ? (float)vim(a) : (float)vre(a);
      else x = (float)vre(a);
    }
    v[q] = x;
  }
  u32x4 h, l;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t h0, l0, h1, l1;
    split2(v[2 * q], h0, l0);
    split2(v[2 * q + 1], h1, l1);
    h[q] = h0 | (h1 << 16);
    l[q] = l0 | (l1 << 16);
  }
  *reinterpret_cast<u32x4*>(hi + row * ldp + k8) = h;
  *reinterpret_cast<u32x4*>(lo + row * ldp + k8) = l;
}

// Planes of the transpose: output row j (< K) holds source column j, its K'
// running over source rows (2 per row for complex data), zero from the real
// extent to ldp.  64 x 64 entry tiles through LDS; grid (ceil(ldp / (64 E)),
// ceil(K / 64)).  The transpose is not conjugated (the GEMM conjugates).
template <typename T>
__global__ void __launch_bounds__(256) k_planes_t(const T* __restrict__ A, int64_t lda, int64_t M, int64_t K,
                                                  uint16_t* __restrict__ hi, uint16_t* __restrict__ lo,
                                                  int64_t ldp) {
  constexpr int E = Elem<T>::cplx ? 2 : 1;
  __shared__ float tile[64][64 * E + 1];  // [source col][source row * E + part]
  const int64_t i0 = (int64_t)blockIdx.x * 64;  // source rows
  const int64_t j0 = (int64_t)blockIdx.y * 64;  // source cols
  const int t = threadIdx.x;
  // read: 64 rows x 64 entries, entry index fastest
  for (int q = t; q < 64 * 64; q += 256) {
    const int r = q / 64, cc = q % 64;
    const int64_t i = i0 + r, j = j0 + cc;
    T a{};
    if (i < M && j < K) a = A[i * lda + j];
    if constexpr (E == 2) {
      tile[cc][2 * r] = (float)vre(a);
      tile[cc][2 * r + 1] = (float)vim(a);
    } else {
      tile[cc][r] = (float)vre(a);
    }
  }
  __syncthreads();
  // write: output rows j0 .. j0+63, K' = E*i0 .. E*i0 + 64E; 8 values per thread
  constexpr int PER_ROW = 64 * E / 8;
  for (int q = t; q < 64 * PER_ROW; q += 256) {
    const int cc = q / PER_ROW, seg = q % PER_ROW;
    const int64_t j = j0 + cc;
    const int64_t k8 = E * i0 + 8 * seg;
    if (j >= K || k8 >= ldp) continue;
    u32x4 h, l;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      uint32_t h0, l0, h1, l1;
      split2(tile[cc][8 * seg + 2 * u], h0, l0);
      split2(tile[cc][8 * seg + 2 * u + 1], h1, l1);
      h[u] = h0 | (h1 << 16);
      l[u] = l0 | (l1 << 16);
    }
    *reinterpret_cast<u32x4*>(hi + j * ldp + k8) = h;
    *reinterpret_cast<u32x4*>(lo + j * ldp + k8) = l;
  }
}

// ---------------------------------------------------------------------------
// k_gemm_bf: C (M x N') = L (M x K') B^ (K' x N') on split BF16 planes.
// Workgroup: 4 waves x 32 rows; all N' = 16 NT columns; K' range of one split
// (blockIdx.y) in chunks of 64.  The right operand's compact columns are
// staged per chunk in LDS already expanded to the real block form.
// MODE 0: FP32 partials Cp[(split * N' + c') * ldc + row].
// MODE 1: compact BF16 planes of C (complex column c interleaved re/im along
//         K' = E * row + part), for the next product's right operand.
constexpr int kBfKc = 64;
constexpr int kBfRows = 128;
constexpr int kBfStride = 72;  // bf16 per staged column: 64 + 8 (bank spread)

template <bool CPLX, bool CONJ, int NT, int MODE>
__global__ void __launch_bounds__(256, 2) k_gemm_bf(BfGemmArgs g) {
  constexpr int NCOL = NT * 16;             // real (expanded) columns
  constexpr int KCOL = CPLX ? NCOL / 2 : NCOL;  // compact columns
  extern __shared__ unsigned char smem_raw[];
  // [buf][plane][NCOL][kBfStride]
  uint16_t* Bs = reinterpret_cast<uint16_t*>(smem_raw);
  constexpr int BUF = 2 * NCOL * kBfStride;
  if (g.flag && *g.flag) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int rl = lane & 15, grp = lane >> 4;
  const int64_t k_begin = (int64_t)blockIdx.y * g.ks;
  const int64_t k_end = k_begin + g.ks < g.Kp ? k_begin + g.ks : g.Kp;
  const int nch = k_end > k_begin ? (int)((k_end - k_begin) / kBfKc) : 0;
  const int64_t row0 = (int64_t)blockIdx.x * kBfRows + wv * 32;

  const uint16_t* ap[2][2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    int64_t r = row0 + 16 * mt + rl;
    if (r > g.M - 1) r = g.M - 1;
    ap[mt][0] = g.Ahi + r * g.lda + 16 * grp;
    ap[mt][1] = g.Alo + r * g.lda + 16 * grp;
  }
  // staging units: 16 B of one compact column and plane
  constexpr int UNITS = KCOL * 2 * (kBfKc / 8);
  constexpr int UPT = (UNITS + 255) / 256;

  f32x4 acc[2][NT];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[mt][t] = f32x4{0.f, 0.f, 0.f, 0.f};

  u32x4 a_cur[2][2][2], a_nxt[2][2][2], b_nxt[UPT];
  auto load_a = [&](int ch, u32x4 (&dst)[2][2][2]) {
    const int64_t k = k_begin + (int64_t)ch * kBfKc;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int pl = 0; pl < 2; ++pl) {
        const u32x4* p = reinterpret_cast<const u32x4*>(ap[mt][pl] + k);
        dst[mt][pl][0] = p[0];
        dst[mt][pl][1] = p[1];
      }
  };
  auto load_b = [&](int ch) {
    const int64_t k = k_begin + (int64_t)ch * kBfKc;
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int u = tid + 256 * i;
      u32x4 v = u32x4{0u, 0u, 0u, 0u};
      if (u < UNITS) {
        const int pl = u / (KCOL * 8), col = (u / 8) % KCOL, q = u % 8;
        if (col < g.kc) v = *reinterpret_cast<const u32x4*>((pl ? g.Blo : g.Bhi) + col * g.ldb + k + 8 * q);
      }
      b_nxt[i] = v;
    }
  };
  auto store_b = [&](int buf) {
    uint16_t* base = Bs + buf * BUF;
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int u = tid + 256 * i;
      if (u >= UNITS) continue;
      const int pl = u / (KCOL * 8), col = (u / 8) % KCOL, q = u % 8;
      const u32x4 v = b_nxt[i];
      if constexpr (CPLX) {
        // column 2c: (br, -bi) [conj: (br, bi)]; column 2c+1: (bi, br) [conj: (bi, -br)]
        u32x4 e, o;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const uint32_t x = v[w];
          const uint32_t sw = (x >> 16) | (x << 16);
          e[w] = CONJ ? x : (x ^ 0x80000000u);
          o[w] = CONJ ? (sw ^ 0x80000000u) : sw;
        }
        *reinterpret_cast<u32x4*>(base + (pl * NCOL + 2 * col) * kBfStride + 8 * q) = e;
        *reinterpret_cast<u32x4*>(base + (pl * NCOL + 2 * col + 1) * kBfStride + 8 * q) = o;
      } else {
        *reinterpret_cast<u32x4*>(base + (pl * NCOL + col) * kBfStride + 8 * q) = v;
      }
    }
  };

  if (nch > 0) {
    load_a(0, a_cur);
    load_b(0);
    store_b(0);
    if (nch > 1) {
      load_a(1, a_nxt);
      load_b(1);
    }
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const uint16_t* bb = Bs + (ch & 1) * BUF;
    // issue order: for a group of up to 2 column tiles, the hi*hi products of
    // all (row tile, column tile) pairs, then hi*lo, then lo*hi, so that
    // consecutive matrix-core instructions accumulate into different tiles
    constexpr int TG = NT < 2 ? NT : 2;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int t0 = 0; t0 < NT; t0 += TG) {
        bf16x8 bh[TG], bl[TG];
#pragma unroll
        for (int tt = 0; tt < TG; ++tt) {
          const int c = 16 * (t0 + tt) + rl;
          bh[tt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(bb + c * kBfStride + 16 * grp + 8 * s));
          bl[tt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(bb + (NCOL + c) * kBfStride + 16 * grp + 8 * s));
        }
#pragma unroll
        for (int pass = 0; pass < 3; ++pass) {
#pragma unroll
          for (int tt = 0; tt < TG; ++tt)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
              const bf16x8 a = __builtin_bit_cast(bf16x8, a_cur[mt][pass == 2 ? 1 : 0][s]);
              const bf16x8 b = pass == 1 ? bl[tt] : bh[tt];
              acc[mt][t0 + tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[mt][t0 + tt], 0, 0, 0);
            }
        }
      }
    }
    if (ch + 1 < nch) {
      store_b((ch + 1) & 1);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int pl = 0; pl < 2; ++pl) {
          a_cur[mt][pl][0] = a_nxt[mt][pl][0];
          a_cur[mt][pl][1] = a_nxt[mt][pl][1];
        }
      if (ch + 2 < nch) {
        load_a(ch + 2, a_nxt);
        load_b(ch + 2);
      }
    }
    __syncthreads();
  }

  // epilogue
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int64_t rb = row0 + 16 * mt + 4 * grp;  // rows rb .. rb+3
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int cp = 16 * t + rl;  // real column
      const f32x4 v = acc[mt][t];
      if constexpr (MODE == 0) {
        float* dst = g.Cp + ((int64_t)blockIdx.y * NCOL + cp) * g.ldc + rb;
        if (rb + 3 < g.M) {
          *reinterpret_cast<f32x4*>(dst) = v;
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (rb + q < g.M) dst[q] = v[q];
        }
      } else if constexpr (CPLX) {
        // lanes 2c' (Re) and 2c'+1 (Im) of one compact column: swap values,
        // the even lane stores the hi plane and the odd lane the lo plane of
        // the 4 complex rows
        float other[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) other[q] = dpp<kDppXor1>(v[q]);
        const bool odd = lane & 1;
        const int col = cp >> 1;
        u32x4 w;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float re = odd ? other[q] : v[q];
          const float im = odd ? v[q] : other[q];
          uint32_t hr, lr, hi_, li;
          split2(re, hr, lr);
          split2(im, hi_, li);
          w[q] = odd ? (lr | (li << 16)) : (hr | (hi_ << 16));
        }
        if (col < g.kc) {
          uint16_t* dst = (odd ? g.Olo : g.Ohi) + col * g.ldo + 2 * rb;
          if (rb + 3 < g.M) {
            *reinterpret_cast<u32x4*>(dst) = w;
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (rb + q < g.M) reinterpret_cast<uint32_t*>(dst)[q] = w[q];
          }
        }
      } else {
        const int col = cp;
        uint32_t h[4], l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) split2(v[q], h[q], l[q]);
        if (col < g.kc) {
          uint16_t* dh = g.Ohi + col * g.ldo + rb;
          uint16_t* dl = g.Olo + col * g.ldo + rb;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (rb + q < g.M) {
              dh[q] = (uint16_t)h[q];
              dl[q] = (uint16_t)l[q];
            }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// k_gemm_d: FP64 C (M x N') = op(L) (M x K) B^ (K x N'), left entries of type
// T (promoted to FP64), right operand compact FP64 columns (cd or double).
// TRANS: L is stored transposed (K x M row-major, ld lda), read along its
// stored rows.  CONJ: op = complex conjugate.  tri = 1: L[r][k] = 0 for
// k < r (upper triangular; the K range starts at the workgroup's first row);
// tri = 2: L[r][k] = 0 for k > r.  Workgroup: 4 waves x 32 rows, chunks of 16
// K entries (4 per lane group).
// MODE 0: FP64 partials Cp[(split * N' + c') * ldc + row].
// MODE 1: compact FP64 columns O[c * ldo + row] (complex for complex T).
constexpr int kDKc = 16;
constexpr int kDRows = 128;

template <typename T, typename BS, bool TRANS, bool CONJ, int NT, int MODE>
__device__ __forceinline__ void k_gemm_d_body(const Bk bk, DGemmArgs g) {
  constexpr bool CPLX = Elem<T>::cplx;
  using BT = typename std::conditional<CPLX, cd, double>::type;
  constexpr int NCOL = NT * 16;
  constexpr int KCOL = CPLX ? NCOL / 2 : NCOL;
  __shared__ BT Bs[2][KCOL][kDKc + 1];
  // bk.z: block of KCOL right-hand columns starting at c0
  const int64_t c0 = (int64_t)bk.z * KCOL;
  const int kcz = g.kc - c0 < KCOL ? (int)(g.kc - c0) : KCOL;
  const int64_t wg_row0 = (int64_t)bk.x * kDRows;
  // Hermitian product: only tiles that reach the upper triangle
  if (g.herm && wg_row0 > c0 + KCOL - 1) return;
  if (g.flag && *g.flag) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int rl = lane & 15, grp = lane >> 4;
  const int64_t row0 = wg_row0 + wv * 32;
  int64_t k_begin = (int64_t)bk.y * g.ks;
  int64_t k_end = k_begin + g.ks < g.K ? k_begin + g.ks : g.K;
  if (g.tri == 1) {
    const int64_t lo = (wg_row0 / kDKc) * kDKc;
    if (k_begin < lo) k_begin = lo;
  } else if (g.tri == 2) {
    const int64_t hi = wg_row0 + kDRows;
    if (k_end > hi) k_end = hi;
  }
  const int nch = k_end > k_begin ? (int)((k_end - k_begin + kDKc - 1) / kDKc) : 0;
  const T* L = reinterpret_cast<const T*>(g.A);
  const BS* B = reinterpret_cast<const BS*>(g.B) + c0 * g.ldb;

  int64_t rows[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    int64_t r = row0 + 16 * mt + rl;
    rows[mt] = r > g.M - 1 ? g.M - 1 : r;
  }
  f64x4 acc[2][NT];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[mt][t] = f64x4{0.0, 0.0, 0.0, 0.0};

  // left entries of lane group grp in a chunk at k: entry u is k + 4 grp + u
  // (row-major L: a contiguous run) or k + 4 u + grp (transposed L: 16
  // consecutive rows of one stored row per group)
  auto kidx = [&](int u) { return TRANS ? 4 * u + grp : 4 * grp + u; };
  T a_cur[2][4], a_nxt[2][4];
  auto load_a = [&](int ch, T (&dst)[2][4]) {
    const int64_t k = k_begin + (int64_t)ch * kDKc;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t kk = k + kidx(u);
        T v{};
        if (kk < k_end) v = TRANS ? L[kk * g.lda + rows[mt]] : L[rows[mt] * g.lda + kk];
        dst[mt][u] = v;
      }
  };
  constexpr int UNITS = KCOL * kDKc;
  constexpr int UPT = (UNITS + 255) / 256;
  BT b_nxt[UPT];
  auto load_b = [&](int ch) {
    const int64_t k = k_begin + (int64_t)ch * kDKc;
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int u = tid + 256 * i;
      BT v{};
      if (u < UNITS) {
        const int col = u / kDKc, q = u % kDKc;
        if (col < kcz && k + q < k_end) {
          const BS e = B[col * g.ldb + k + q];
          v = vconv<BT>(e);
        }
      }
      b_nxt[i] = v;
    }
  };
  auto store_b = [&](int buf) {
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int u = tid + 256 * i;
      if (u < UNITS) Bs[buf][u / kDKc][u % kDKc] = b_nxt[i];
    }
  };
  const bool odd = lane & 1;

  if (nch > 0) {
    load_a(0, a_cur);
    load_b(0);
    store_b(0);
    if (nch > 1) {
      load_a(1, a_nxt);
      load_b(1);
    }
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kl = kidx(u);
      if constexpr (CPLX) {
        // expanded column: even (br, -bi) / conj (br, bi); odd (bi, br) / conj (bi, -br).
        // All real parts first, then all imaginary parts: consecutive
        // instructions accumulate into different tiles.
        double b_re[NT], b_im[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const cd b = Bs[buf][8 * t + (rl >> 1)][kl];
          b_re[t] = odd ? b.im : b.re;
          b_im[t] = CONJ ? (odd ? -b.re : b.im) : (odd ? b.re : -b.im);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int mt = 0; mt < 2; ++mt)
            acc[mt][t] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)vre(a_cur[mt][u]), b_re[t], acc[mt][t], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int mt = 0; mt < 2; ++mt)
            acc[mt][t] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)vim(a_cur[mt][u]), b_im[t], acc[mt][t], 0, 0, 0);
      } else {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const double b = Bs[buf][16 * t + rl][kl];
#pragma unroll
          for (int mt = 0; mt < 2; ++mt)
            acc[mt][t] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)vre(a_cur[mt][u]), b, acc[mt][t], 0, 0, 0);
        }
      }
    }
    if (ch + 1 < nch) {
      store_b(buf ^ 1);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int u = 0; u < 4; ++u) a_cur[mt][u] = a_nxt[mt][u];
      if (ch + 2 < nch) {
        load_a(ch + 2, a_nxt);
        load_b(ch + 2);
      }
    }
    __syncthreads();
  }

  // f64 accumulator layout: lane l holds column l%16, rows 4 v + l/16
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int64_t rb = row0 + 16 * mt + grp;  // rows rb + 4 v
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int cp = 16 * t + rl;
      const f64x4 v = acc[mt][t];
      if constexpr (MODE == 0) {
        double* dst = g.Cp + (((int64_t)bk.z * bk.gy + bk.y) * NCOL + cp) * g.ldc + rb;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (rb + 4 * q < g.M) dst[4 * q] = v[q];
      } else if constexpr (CPLX) {
        double other[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) other[q] = dpp<kDppXor1>(v[q]);
        const int col = cp >> 1;
        // even lane: rows rb, rb+4; odd lane: rows rb+8, rb+12
        cd* dst = reinterpret_cast<cd*>(g.O) + (c0 + col) * g.ldo;
        if (col < kcz) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int q = odd ? 2 + h : h;
            const double re = odd ? other[q] : v[q];
            const double im = odd ? v[q] : other[q];
            if (rb + 4 * q < g.M) dst[rb + 4 * q] = cd{re, im};
          }
        }
      } else {
        const int col = cp;
        double* dst = reinterpret_cast<double*>(g.O) + (c0 + col) * g.ldo;
        if (col < kcz) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (rb + 4 * q < g.M) dst[rb + 4 * q] = v[q];
        }
      }
    }
  }
}
template <typename T, typename BS, bool TRANS, bool CONJ, int NT, int MODE>
__global__ void __launch_bounds__(256) k_gemm_d(DGemmArgs g) {
  k_gemm_d_body<T, BS, TRANS, CONJ, NT, MODE>(bk_hw(), g);
}

// ---------------------------------------------------------------------------
// Sum of split partials (column-major real columns) into compact FP64
// columns: out[c][r] = sum_s C_s[r][c] (or src[c][r] - sum).  grid
// (ceil(M / 256), kc).
template <typename P, typename W>
__global__ void __launch_bounds__(256) k_blk_reduce(const P* __restrict__ Cp, int splits, int64_t ldc, int ncol,
                                                    int64_t M, const W* __restrict__ src, int64_t lds,
                                                    W* __restrict__ out, int64_t ldo,
                                                    const int32_t* __restrict__ flag) {
  if (flag && *flag) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= M) return;
  if constexpr (VT<W>::cplx) {
    double re = 0.0, im = 0.0;
    for (int s = 0; s < splits; ++s) {
      re += (double)Cp[((int64_t)s * ncol + 2 * c) * ldc + r];
      im += (double)Cp[((int64_t)s * ncol + 2 * c + 1) * ldc + r];
    }
    W v = cd{re, im};
    if (src) v = vsub(src[c * lds + r], v);
    out[c * ldo + r] = v;
  } else {
    double s_ = 0.0;
    for (int s = 0; s < splits; ++s) s_ += (double)Cp[((int64_t)s * ncol + c) * ldc + r];
    W v = s_;
    if (src) v = src[c * lds + r] - v;
    out[c * ldo + r] = v;
  }
}

// ---------------------------------------------------------------------------
// Block CG: one workgroup per right-hand side column.
__device__ inline void col_pair_sums(double& a, double& b, double* red) {
  a = block_sum(a, red);
  b = block_sum(b, red + 4);
}

// Start of a refinement step for column c: certificate of y_out from its FP64
// residual rr and s = X* rr (rule R at eps_outer / 2, as in the one-column
// path); then y = 0, r = rr, rho0 = rho = ||s||^2.
template <typename W>
__global__ void __launch_bounds__(256) k_blk_outer(int64_t m, const W* __restrict__ b, int64_t ldb,
                                                   const W* __restrict__ rr, const W* __restrict__ s,
                                                   const W* __restrict__ y_out, W* __restrict__ y,
                                                   W* __restrict__ r, BlkState* __restrict__ st) {
  __shared__ double red[8];
  const int c = blockIdx.x;
  BlkCol& col = st->col[c];
  if (col.outer_done) return;
  const W* bc = b + c * ldb;
  double rho = 0.0, xi = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
    rho += vabs2(s[c * m + i]);
    xi += vre(vcmul(y_out[c * m + i], vsub(bc[i], rr[c * m + i])));
  }
  col_pair_sums(rho, xi, red);
  const double e = 0.5 * st->eps_outer;
  const double tol = e / (1.0 + e);
  int od = 0, status = col.status;
  if (!(isfinite(rho) && isfinite(xi))) {
    od = 1;
    status = 4;
  } else if (rho <= tol * tol * xi || rho == 0.0) {
    od = 1;
  } else if (col.refine >= st->max_refine) {
    od = 1;
    status = 2;
  }
  if (!od) {
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
      y[c * m + i] = vzero<W>();
      r[c * m + i] = rr[c * m + i];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    col.outer_rho = rho;
    col.outer_xi = xi;
    col.status = status;
    col.outer_done = od;
    col.rho0 = rho;
    col.rho = rho;
    col.inner_it = 0;
    col.inner_done = od;
  }
}

// alpha_c = rho_c / Re(p_c* q_c); y_c += alpha p_c; r_c -= alpha q_c.
template <typename W>
__global__ void __launch_bounds__(256) k_blk_alpha(int64_t m, const W* __restrict__ p, const W* __restrict__ q,
                                                   W* __restrict__ y, W* __restrict__ r,
                                                   BlkState* __restrict__ st) {
  __shared__ double red[4];
  if (st->all_inner_done) return;
  const int c = blockIdx.x;
  BlkCol& col = st->col[c];
  if (col.inner_done) return;
  double pq = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) pq += vre(vcmul(p[c * m + i], q[c * m + i]));
  pq = block_sum(pq, red);
  const double alpha = col.rho / pq;
  if (!(isfinite(alpha) && pq > 0.0)) {
    __syncthreads();
    if (threadIdx.x == 0) {
      col.inner_done = 1;
      col.outer_done = 1;
      col.status = 4;
    }
    return;
  }
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
    y[c * m + i] = vadd(y[c * m + i], vscale(p[c * m + i], alpha));
    r[c * m + i] = vsub(r[c * m + i], vscale(q[c * m + i], alpha));
  }
}

// start: p = z.  iteration: rho' = ||s||^2, inner stopping test
// rho' <= eps_inner^2 rho0, beta = rho'/rho, p = z + beta p.  Writes the BF16
// planes of p (column c, K' = E i + part) for the next A* p product.
template <typename W>
__global__ void __launch_bounds__(256) k_blk_beta(int64_t m, int start, const W* __restrict__ s,
                                                  const W* __restrict__ z, W* __restrict__ p,
                                                  uint16_t* __restrict__ phi, uint16_t* __restrict__ plo,
                                                  int64_t ldp, BlkState* __restrict__ st) {
  __shared__ double red[4];
  __shared__ int stop_s;
  __shared__ double beta_s;
  const int c = blockIdx.x;
  BlkCol& col = st->col[c];
  if (start) {
    if (col.outer_done) return;
  } else {
    if (st->all_inner_done || col.inner_done) return;
  }
  double beta = 0.0;
  if (!start) {
    double rho = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) rho += vabs2(s[c * m + i]);
    rho = block_sum(rho, red);
    if (threadIdx.x == 0) {
      const int it = col.inner_it + 1;
      int stop = 0;
      if (!isfinite(rho)) {
        stop = 1;
        col.status = 4;
        col.outer_done = 1;
      } else if (rho <= st->eps_inner * st->eps_inner * col.rho0 || it >= st->max_iter) {
        stop = 1;
      }
      beta_s = rho / col.rho;
      col.inner_it = it;
      col.iters += 1;
      col.rho_prev = col.rho;
      col.rho = rho;
      if (stop) col.inner_done = 1;
      stop_s = stop;
    }
    __syncthreads();
    if (stop_s) return;
    beta = beta_s;
  }
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
    W v = z[c * m + i];
    if (!start) v = vadd(v, vscale(p[c * m + i], beta));
    p[c * m + i] = v;
    if constexpr (VT<W>::cplx) {
      uint32_t hr, lr, hi_, li;
      split2((float)v.re, hr, lr);
      split2((float)v.im, hi_, li);
      reinterpret_cast<uint32_t*>(phi + c * ldp)[i] = hr | (hi_ << 16);
      reinterpret_cast<uint32_t*>(plo + c * ldp)[i] = lr | (li << 16);
    } else {
      uint32_t h, l;
      split2((float)v, h, l);
      phi[c * ldp + i] = (uint16_t)h;
      plo[c * ldp + i] = (uint16_t)l;
    }
  }
}

// all_inner_done / all_outer_done over the kc columns (one wave).
__global__ void k_blk_flag(BlkState* __restrict__ st) {
  const int c = threadIdx.x;
  const bool live = c < st->kc;
  const bool in_done = !live || st->col[c].inner_done || st->col[c].outer_done;
  const bool out_done = !live || st->col[c].outer_done;
  const bool all_in = __all(in_done), all_out = __all(out_done);
  if (c == 0) {
    st->all_inner_done = all_in ? 1 : 0;
    st->all_outer_done = all_out ? 1 : 0;
  }
}

// y_out += y for columns still refining; counts the refinement step.
template <typename W>
__global__ void __launch_bounds__(256) k_blk_refine(int64_t m, W* __restrict__ y_out, const W* __restrict__ y,
                                                    BlkState* __restrict__ st) {
  const int c = blockIdx.y;
  BlkCol& col = st->col[c];
  if (col.outer_done) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) y_out[c * m + i] = vadd(y_out[c * m + i], y[c * m + i]);
  if (blockIdx.x == 0 && threadIdx.x == 0) col.refine += 1;
}

// Fill of 16-byte units (zeroing buffers without a memset node).
__global__ void k_fill16(u32x4* __restrict__ p, int64_t n16) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) p[i] = u32x4{0u, 0u, 0u, 0u};
}

// ---------------------------------------------------------------------------
// launchers

int bf_nt(bool cplx, int kc) {
  const int ncol = cplx ? 2 * kc : kc;
  return ncol <= 16 ? 1 : ncol <= 32 ? 2 : ncol <= 64 ? 4 : 8;
}

int64_t bf_ktile() { return kBfKc; }

hipError_t launch_planes(int dtype, const void* A, int64_t lda, int64_t M, int64_t K, bool trans, uint16_t* hi,
                         uint16_t* lo, int64_t ldp, hipStream_t st) {
  if (ldp % 8 != 0) return hipErrorInvalidValue;
  if (!trans) {
    const dim3 grid((unsigned)ceil_div(ldp, 8 * 256), (unsigned)M);
    switch (dtype) {
      case 0: hipLaunchKernelGGL(k_planes<cd>, grid, dim3(256), 0, st, (const cd*)A, lda, M, K, hi, lo, ldp); break;
      case 1: hipLaunchKernelGGL(k_planes<cf>, grid, dim3(256), 0, st, (const cf*)A, lda, M, K, hi, lo, ldp); break;
      case 2: hipLaunchKernelGGL(k_planes<double>, grid, dim3(256), 0, st, (const double*)A, lda, M, K, hi, lo, ldp); break;
      case 3: hipLaunchKernelGGL(k_planes<float>, grid, dim3(256), 0, st, (const float*)A, lda, M, K, hi, lo, ldp); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const int E = (dtype == 0 || dtype == 1) ? 2 : 1;
    const dim3 grid((unsigned)ceil_div(ldp, 64 * E), (unsigned)ceil_div(K, 64));
    switch (dtype) {
      case 0: hipLaunchKernelGGL(k_planes_t<cd>, grid, dim3(256), 0, st, (const cd*)A, lda, M, K, hi, lo, ldp); break;
      case 1: hipLaunchKernelGGL(k_planes_t<cf>, grid, dim3(256), 0, st, (const cf*)A, lda, M, K, hi, lo, ldp); break;
      case 2: hipLaunchKernelGGL(k_planes_t<double>, grid, dim3(256), 0, st, (const double*)A, lda, M, K, hi, lo, ldp); break;
      case 3: hipLaunchKernelGGL(k_planes_t<float>, grid, dim3(256), 0, st, (const float*)A, lda, M, K, hi, lo, ldp); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <bool CPLX, bool CONJ, int NT, int MODE>
hipError_t bf_go(const BfGemmArgs& a, int splits, hipStream_t st) {
  constexpr int NCOL = NT * 16;
  const size_t lds = (size_t)2 * 2 * NCOL * kBfStride * sizeof(uint16_t);
  auto kern = k_gemm_bf<CPLX, CONJ, NT, MODE>;
  static const hipError_t attr =
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  const dim3 grid((unsigned)ceil_div(a.M, kBfRows), (unsigned)splits);
  hipLaunchKernelGGL(kern, grid, dim3(256), lds, st, a);
  return hipGetLastError();
}

template <bool CPLX, bool CONJ, int MODE>
hipError_t bf_nt_go(const BfGemmArgs& a, int nt, int splits, hipStream_t st) {
  switch (nt) {
    case 1: return bf_go<CPLX, CONJ, 1, MODE>(a, splits, st);
    case 2: return bf_go<CPLX, CONJ, 2, MODE>(a, splits, st);
    case 4: return bf_go<CPLX, CONJ, 4, MODE>(a, splits, st);
    case 8: return bf_go<CPLX, CONJ, 8, MODE>(a, splits, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_bf(bool cplx, bool conj, int mode, const BfGemmArgs& a, int splits, hipStream_t st) {
  if (a.Kp % kBfKc != 0 || a.ks % kBfKc != 0 || a.lda % 8 != 0 || a.ldb % 8 != 0 || a.kc < 1 || a.kc > 64 ||
      splits < 1 || (int64_t)splits * a.ks < a.Kp)
    return hipErrorInvalidValue;
  if (mode == 0 && a.ldc % 4 != 0) return hipErrorInvalidValue;
  if (mode == 1 && splits != 1) return hipErrorInvalidValue;
  if (mode == 1 && a.ldo % 8 != 0) return hipErrorInvalidValue;
  const int nt = bf_nt(cplx, a.kc);
  if (cplx) {
    if (conj) return mode ? bf_nt_go<true, true, 1>(a, nt, splits, st) : bf_nt_go<true, true, 0>(a, nt, splits, st);
    return mode ? bf_nt_go<true, false, 1>(a, nt, splits, st) : bf_nt_go<true, false, 0>(a, nt, splits, st);
  }
  return mode ? bf_nt_go<false, false, 1>(a, nt, splits, st) : bf_nt_go<false, false, 0>(a, nt, splits, st);
}

template <typename T, bool TRANS, bool CONJ, int MODE>
hipError_t d_nt_go(const DGemmArgs& a, int nt, int splits, hipStream_t st) {
  using W = typename std::conditional<Elem<T>::cplx, cd, double>::type;
  const dim3 grid((unsigned)ceil_div(a.M, kDRows), (unsigned)splits);
  switch (nt) {
    case 1: hipLaunchKernelGGL((k_gemm_d<T, W, TRANS, CONJ, 1, MODE>), grid, dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_gemm_d<T, W, TRANS, CONJ, 2, MODE>), grid, dim3(256), 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_gemm_d<T, W, TRANS, CONJ, 4, MODE>), grid, dim3(256), 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_gemm_d<T, W, TRANS, CONJ, 8, MODE>), grid, dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t d_go(bool trans, bool conj, int mode, const DGemmArgs& a, int nt, int splits, hipStream_t st) {
  if (trans) {
    if (conj) return mode ? d_nt_go<T, true, true, 1>(a, nt, splits, st) : d_nt_go<T, true, true, 0>(a, nt, splits, st);
    return mode ? d_nt_go<T, true, false, 1>(a, nt, splits, st) : d_nt_go<T, true, false, 0>(a, nt, splits, st);
  }
  if (conj) return mode ? d_nt_go<T, false, true, 1>(a, nt, splits, st) : d_nt_go<T, false, true, 0>(a, nt, splits, st);
  return mode ? d_nt_go<T, false, false, 1>(a, nt, splits, st) : d_nt_go<T, false, false, 0>(a, nt, splits, st);
}

hipError_t launch_gemm_d(int dtype, bool trans, bool conj, int mode, const DGemmArgs& a, int splits, hipStream_t st) {
  if (a.kc < 1 || a.kc > 64 || a.herm || splits < 1 || (int64_t)splits * a.ks < a.K || a.ks % kDKc != 0)
    return hipErrorInvalidValue;
  if (mode == 1 && splits != 1) return hipErrorInvalidValue;
  const bool cplx = dtype == 0 || dtype == 1;
  const int nt = bf_nt(cplx, a.kc);
  switch (dtype) {
    case 0: return d_go<cd>(trans, conj, mode, a, nt, splits, st);
    case 1: return d_go<cf>(trans, conj, mode, a, nt, splits, st);
    case 2: return d_go<double>(trans, false, mode, a, nt, splits, st);
    case 3: return d_go<float>(trans, false, mode, a, nt, splits, st);
  }
  return hipErrorInvalidValue;
}

int gemm_ncol(bool cplx, int kc) { return 16 * bf_nt(cplx, kc); }

hipError_t launch_blk_reduce(bool cplx, bool f32, const void* Cp, int splits, int64_t ldc, int ncol, int64_t M,
                             int kc, const void* src, int64_t lds, void* out, int64_t ldo, const int32_t* flag,
                             hipStream_t st) {
  const dim3 grid((unsigned)ceil_div(M, 256), (unsigned)kc);
  if (cplx) {
    if (f32)
      hipLaunchKernelGGL((k_blk_reduce<float, cd>), grid, dim3(256), 0, st, (const float*)Cp, splits, ldc, ncol, M,
                         (const cd*)src, lds, (cd*)out, ldo, flag);
    else
      hipLaunchKernelGGL((k_blk_reduce<double, cd>), grid, dim3(256), 0, st, (const double*)Cp, splits, ldc, ncol,
                         M, (const cd*)src, lds, (cd*)out, ldo, flag);
  } else {
    if (f32)
      hipLaunchKernelGGL((k_blk_reduce<float, double>), grid, dim3(256), 0, st, (const float*)Cp, splits, ldc, ncol,
                         M, (const double*)src, lds, (double*)out, ldo, flag);
    else
      hipLaunchKernelGGL((k_blk_reduce<double, double>), grid, dim3(256), 0, st, (const double*)Cp, splits, ldc,
                         ncol, M, (const double*)src, lds, (double*)out, ldo, flag);
  }
  return hipGetLastError();
}

hipError_t launch_blk_outer(bool cplx, int kc, int64_t m, const void* b, int64_t ldb, const void* rr, const void* s,
                            const void* y_out, void* y, void* r, BlkState* state, hipStream_t st) {
  if (cplx)
    hipLaunchKernelGGL(k_blk_outer<cd>, dim3(kc), dim3(256), 0, st, m, (const cd*)b, ldb, (const cd*)rr,
                       (const cd*)s, (const cd*)y_out, (cd*)y, (cd*)r, state);
  else
    hipLaunchKernelGGL(k_blk_outer<double>, dim3(kc), dim3(256), 0, st, m, (const double*)b, ldb,
                       (const double*)rr, (const double*)s, (const double*)y_out, (double*)y, (double*)r, state);
  return hipGetLastError();
}

hipError_t launch_blk_alpha(bool cplx, int kc, int64_t m, const void* p, const void* q, void* y, void* r,
                            BlkState* state, hipStream_t st) {
  if (cplx)
    hipLaunchKernelGGL(k_blk_alpha<cd>, dim3(kc), dim3(256), 0, st, m, (const cd*)p, (const cd*)q, (cd*)y, (cd*)r,
                       state);
  else
    hipLaunchKernelGGL(k_blk_alpha<double>, dim3(kc), dim3(256), 0, st, m, (const double*)p, (const double*)q,
                       (double*)y, (double*)r, state);
  return hipGetLastError();
}

hipError_t launch_blk_beta(bool cplx, int kc, int64_t m, int start, const void* s, const void* z, void* p,
                           uint16_t* phi, uint16_t* plo, int64_t ldp, BlkState* state, hipStream_t st) {
  if (cplx)
    hipLaunchKernelGGL(k_blk_beta<cd>, dim3(kc), dim3(256), 0, st, m, start, (const cd*)s, (const cd*)z, (cd*)p,
                       phi, plo, ldp, state);
  else
    hipLaunchKernelGGL(k_blk_beta<double>, dim3(kc), dim3(256), 0, st, m, start, (const double*)s,
                       (const double*)z, (double*)p, phi, plo, ldp, state);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_blk_flag, dim3(1), dim3(64), 0, st, state);
  return hipGetLastError();
}

hipError_t launch_blk_flag(BlkState* state, hipStream_t st) {
  hipLaunchKernelGGL(k_blk_flag, dim3(1), dim3(64), 0, st, state);
  return hipGetLastError();
}

hipError_t launch_blk_refine(bool cplx, int kc, int64_t m, void* y_out, const void* y, BlkState* state,
                             hipStream_t st) {
  const dim3 grid((unsigned)ceil_div(m, 256), (unsigned)kc);
  if (cplx)
    hipLaunchKernelGGL(k_blk_refine<cd>, grid, dim3(256), 0, st, m, (cd*)y_out, (const cd*)y, state);
  else
    hipLaunchKernelGGL(k_blk_refine<double>, grid, dim3(256), 0, st, m, (double*)y_out, (const double*)y, state);
  return hipGetLastError();
}

// Gram matrix G = S* S (m x m, FP64, upper triangle) of the column-major l x m
// sketch S, on the FP64 matrix cores.  Column blocks of 64 (complex) or 128
// (real) run along blockIdx.z; with several splits of the l rows the partials
// Cp[((z * splits + split) * 128 + c') * ldc + row] are folded by
// launch_gram_fold.
template <typename T, int MODE>
hipError_t gram_go(const DGemmArgs& a, int splits, hipStream_t st) {
  constexpr bool C = Elem<T>::cplx;
  const int kb = C ? 64 : 128;
  const dim3 grid((unsigned)ceil_div(a.M, kDRows), (unsigned)splits, (unsigned)ceil_div(a.kc, kb));
  hipLaunchKernelGGL((k_gemm_d<T, T, false, C, 8, MODE>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

int gram_col_block(int dtype) { return (dtype == 0 || dtype == 1) ? 64 : 128; }

hipError_t launch_gram_s(int dtype, const void* S, int64_t lds, int64_t l, int64_t m, void* G, int64_t ldg,
                         double* Cp, int64_t ldc, int splits, int64_t ks, hipStream_t st) {
  DGemmArgs a{};
  a.A = S;
  a.lda = lds;
  a.M = m;
  a.K = l;
  a.B = S;
  a.ldb = lds;
  a.kc = (int)m;
  a.ks = ks;
  a.herm = 1;
  a.Cp = Cp;
  a.ldc = ldc;
  a.O = G;
  a.ldo = ldg;
  if (splits < 1 || (int64_t)splits * ks < l || ks % kDKc != 0) return hipErrorInvalidValue;
  const int mode = splits > 1 ? 0 : 1;
  switch (dtype) {
    case 0: return mode ? gram_go<cd, 1>(a, 1, st) : gram_go<cd, 0>(a, splits, st);
    case 1: return mode ? gram_go<cf, 1>(a, 1, st) : gram_go<cf, 0>(a, splits, st);
    case 2: return mode ? gram_go<double, 1>(a, 1, st) : gram_go<double, 0>(a, splits, st);
    case 3: return mode ? gram_go<float, 1>(a, 1, st) : gram_go<float, 0>(a, splits, st);
  }
  return hipErrorInvalidValue;
}

// G[r][c] = sum over splits (upper triangle r <= c only).  grid (ceil(m/256), m).
template <bool CPLX>
__global__ void __launch_bounds__(256) k_gram_fold(const double* __restrict__ Cp, int splits, int64_t ldc,
                                                   int64_t m, double* __restrict__ G, int64_t ldg) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= m || r > c) return;
  constexpr int KB = CPLX ? 64 : 128;
  const int64_t z = c / KB, cc = c % KB;
  if (CPLX) {
    double re = 0.0, im = 0.0;
    for (int s = 0; s < splits; ++s) {
      const double* base = Cp + ((z * splits + s) * 128) * ldc;
      re += base[(2 * cc) * ldc + r];
      im += base[(2 * cc + 1) * ldc + r];
    }
    G[2 * (c * ldg + r)] = re;
    G[2 * (c * ldg + r) + 1] = im;
  } else {
    double v = 0.0;
    for (int s = 0; s < splits; ++s) v += Cp[((z * splits + s) * 128 + cc) * ldc + r];
    G[c * ldg + r] = v;
  }
}

hipError_t launch_gram_fold(bool cplx, const double* Cp, int splits, int64_t ldc, int64_t m, void* G, int64_t ldg,
                            hipStream_t st) {
  const dim3 grid((unsigned)ceil_div(m, 256), (unsigned)m);
  if (cplx)
    hipLaunchKernelGGL(k_gram_fold<true>, grid, dim3(256), 0, st, Cp, splits, ldc, m, (double*)G, ldg);
  else
    hipLaunchKernelGGL(k_gram_fold<false>, grid, dim3(256), 0, st, Cp, splits, ldc, m, (double*)G, ldg);
  return hipGetLastError();
}


hipError_t launch_fill0(void* p, int64_t bytes, hipStream_t st) {
  if (bytes % 16 != 0 || ((uintptr_t)p & 15) != 0) return hipErrorInvalidValue;
  const int64_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill16, dim3((unsigned)ceil_div(n16, 256)), dim3(256), 0, st, (u32x4*)p, n16);
  return hipGetLastError();
}

// ------------------------------ batched systems -------------------------------
namespace {
// G = S* S of each system (one split, upper tiles only)
template <typename T>
__global__ void __launch_bounds__(256) kb_gram_s(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                 int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  DGemmArgs a{};
  a.A = s.S;
  a.lda = s.l;
  a.M = s.m;
  a.K = s.l;
  a.B = s.S;
  a.ldb = s.l;
  a.kc = (int)s.m;
  a.ks = ceil_div(s.l, kDKc) * kDKc;
  a.herm = 1;
  a.O = s.G;
  a.ldo = s.m;
  const Bk bk = bgrid_local(grid[i], (int)blockIdx.x - grid[i].start);
  if (bk.x * kDRows > bk.z * (Elem<T>::cplx ? 64 : 128) + (Elem<T>::cplx ? 63 : 127)) return;
  k_gemm_d_body<T, T, false, Elem<T>::cplx, 8, 1>(bk, a);
}
}  // namespace

hipError_t launch_b_gram_s(int dtype, const BLaunch& L, hipStream_t st) {
  switch (dtype) {
    case 0: hipLaunchKernelGGL(kb_gram_s<cd>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys); break;
    case 1: hipLaunchKernelGGL(kb_gram_s<cf>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys); break;
    case 2:
      hipLaunchKernelGGL(kb_gram_s<double>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys);
      break;
    case 3:
      hipLaunchKernelGGL(kb_gram_s<float>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mn
