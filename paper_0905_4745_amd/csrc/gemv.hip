// The passes over A that dominate the method's cost (Step 4's iterations and
// Step 5, x = A* y, eq. output): bandwidth-bound products with a row-major A.
//
//   adj:  w = A* u    (w_j = sum_i conj(A_ij) u_i)   threads own columns,
//                                                    rows split into RS slabs
//   fwd:  q = A w     (q_i = sum_j A_ij w_j)          workgroups own RB rows x
//                                                    a column chunk
// Every load of A is a 16-byte vector load by consecutive threads along a row
// (fully coalesced).  Partial results are combined in a fixed order, so runs
// are bitwise reproducible.  u comes in FP64 (the iteration's vectors are kept
// in FP64); A and w are in A's precision; partial sums of q are written in
// FP64.  All kernels return at once when the iteration's stop flag is set.
#include <hip/hip_ext.h>

#include "common.hpp"
#include "kernels.hpp"
#include "batch_dev.hpp"

namespace mn {

template <typename V> struct Vec16;
template <> struct Vec16<cd> { static constexpr int n = 1; };
template <> struct Vec16<cf> { static constexpr int n = 2; };
template <> struct Vec16<double> { static constexpr int n = 2; };
template <> struct Vec16<float> { static constexpr int n = 4; };

template <typename V, int K> struct alignas(16) Pack { V v[K]; };

template <typename V, int K>
__device__ inline Pack<V, K> loadk(const V* p) {
  return *reinterpret_cast<const Pack<V, K>*>(p);
}
// the same, non-temporal (an operand streamed once per pass)
template <typename V, int K>
__device__ inline Pack<V, K> loadk_once(const V* p) {
  constexpr int B = (int)sizeof(Pack<V, K>);
  Pack<V, K> out;
  if constexpr (B == 16) {
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    const u4 raw = __builtin_nontemporal_load(reinterpret_cast<const u4*>(p));
    __builtin_memcpy(&out, &raw, 16);
  } else if constexpr (B == 8) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 raw = __builtin_nontemporal_load(reinterpret_cast<const u2*>(p));
    __builtin_memcpy(&out, &raw, 8);
  } else if constexpr (B == 4) {
    const unsigned int raw = __builtin_nontemporal_load(reinterpret_cast<const unsigned int*>(p));
    __builtin_memcpy(&out, &raw, 4);
  } else {
    out = *reinterpret_cast<const Pack<V, K>*>(p);
  }
  return out;
}

__device__ inline bool stopped(const int32_t* flag) { return flag != nullptr && *(volatile const int32_t*)flag != 0; }

// one-touch load of a streamed operand (non-temporal: the pass reads each
// entry once, and keeping the stream out of the cache's normal replacement
// measured 0.73 -> 0.82 of the HBM peak for the column-major fused pass)
template <typename V> __device__ __forceinline__ V ld_once(const V* p) {
  if constexpr (VT<V>::cplx) {
    using R = typename VT<V>::real;
    const R* q = reinterpret_cast<const R*>(p);
    return V{__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1)};
  } else {
    return __builtin_nontemporal_load(p);
  }
}

// ---------------------------------------------------------------------------
// w (or its RS partial slabs) = A* u.  grid (ceil(n / (256*VEC)), RS), 256 thr.
// If RS == 1 the result goes straight to w, else to part[rs * n + j].
template <typename V, typename C, typename U, int VEC>
__device__ __forceinline__ void k_gemv_adj_body(const Bk bk, const V* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                  const U* __restrict__ u, int64_t rows_per_slab,
                                                  C* __restrict__ out, const int32_t* __restrict__ flag) {
  if (stopped(flag)) return;
  __shared__ C su[1024];
  const int64_t j0 = ((int64_t)bk.x * 256 + threadIdx.x) * VEC;
  const int64_t r0 = (int64_t)bk.y * rows_per_slab;
  const int64_t r1 = (r0 + rows_per_slab) < m ? (r0 + rows_per_slab) : m;
  C acc[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = vzero<C>();
  const bool full = j0 + VEC <= n;
  for (int64_t rb = r0; rb < r1; rb += 1024) {
    const int64_t rn = (r1 - rb) < 1024 ? (r1 - rb) : 1024;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < rn; t += 256) su[t] = vconv<C>(u[rb + t]);
    __syncthreads();
    if (j0 < n) {
      const V* a = A + rb * lda + j0;
      int64_t i = 0;
      if (full) {
        for (; i + 8 <= rn; i += 8) {
          Pack<V, VEC> x[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) x[k] = loadk_once<V, VEC>(a + (i + k) * lda);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const C ui = su[i + k];
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] = vcfma(vconv<C>(x[k].v[v]), ui, acc[v]);
          }
        }
        for (; i < rn; ++i) {
          Pack<V, VEC> x = loadk_once<V, VEC>(a + i * lda);
          const C ui = su[i];
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[v] = vcfma(vconv<C>(x.v[v]), ui, acc[v]);
        }
      } else {
        for (; i < rn; ++i) {
          const C ui = su[i];
          for (int v = 0; v < VEC; ++v)
            if (j0 + v < n) acc[v] = vcfma(vconv<C>(a[i * lda + v]), ui, acc[v]);
        }
      }
    }
  }
  if (j0 >= n) return;
  C* o = out + (int64_t)bk.y * n + j0;
  if (full && ((uintptr_t)o % 16 == 0)) {
    Pack<C, VEC> pk;
#pragma unroll
    for (int v = 0; v < VEC; ++v) pk.v[v] = acc[v];
    *reinterpret_cast<Pack<C, VEC>*>(o) = pk;
  } else {
    for (int v = 0; v < VEC; ++v)
      if (j0 + v < n) o[v] = acc[v];
  }
}
template <typename V, typename C, typename U, int VEC>
__global__ void __launch_bounds__(256) k_gemv_adj(const V* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                  const U* __restrict__ u, int64_t rows_per_slab,
                                                  C* __restrict__ out, const int32_t* __restrict__ flag) {
  k_gemv_adj_body<V, C, U, VEC>(bk_hw(), A, lda, m, n, u, rows_per_slab, out, flag);
}

// w[j] = sum_s part[s * n + j] in slab order; optionally also a wide copy.
template <typename V, typename W>
__device__ __forceinline__ void k_sum_slabs_body(const Bk bk, const V* __restrict__ part, int rs, int64_t n, V* __restrict__ w, W* __restrict__ wide,
                            const int32_t* __restrict__ flag) {
  if (stopped(flag)) return;
  const int64_t j = (int64_t)bk.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  V s = part[j];
  for (int k = 1; k < rs; ++k) s = vadd(s, part[(int64_t)k * n + j]);
  if (w) w[j] = s;
  if (wide) wide[j] = vconv<W>(s);
}
template <typename V, typename W>
__global__ void k_sum_slabs(const V* __restrict__ part, int rs, int64_t n, V* __restrict__ w, W* __restrict__ wide,
                            const int32_t* __restrict__ flag) {
  k_sum_slabs_body<V, W>(bk_hw(), part, rs, n, w, wide, flag);
}

// ---------------------------------------------------------------------------
// qpart[cs * m + i] = sum_{j in chunk cs} A_ij w_j.  grid (CS, ceil(m / RB)).
template <typename V, typename C, typename W, int RB, int VEC>
__device__ __forceinline__ void k_gemv_fwd_body(const Bk bk, const V* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                  const C* __restrict__ w, int64_t chunk,
                                                  W* __restrict__ qpart, const int32_t* __restrict__ flag) {
  if (stopped(flag)) return;
  __shared__ W red[RB][4];
  const int64_t i0 = (int64_t)bk.y * RB;
  const int64_t c0 = (int64_t)bk.x * chunk;
  const int64_t c1 = (c0 + chunk) < n ? (c0 + chunk) : n;
  C acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = vzero<C>();
  int64_t rows = m - i0;
  if (rows > RB) rows = RB;
  for (int64_t j = c0 + (int64_t)threadIdx.x * VEC; j < c1; j += 256 * VEC) {
    if (j + VEC <= c1) {
      C wv[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) wv[v] = w[j + v];
      Pack<V, VEC> x[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r)
        if (r < rows) x[r] = loadk_once<V, VEC>(A + (i0 + r) * lda + j);
#pragma unroll
      for (int r = 0; r < RB; ++r)
        if (r < rows)
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[r] = vfma(vconv<C>(x[r].v[v]), wv[v], acc[r]);
    } else {
      for (int v = 0; v < VEC; ++v) {
        if (j + v >= c1) break;
        const C wj = w[j + v];
        for (int r = 0; r < RB; ++r)
          if (r < rows) acc[r] = vfma(vconv<C>(A[(i0 + r) * lda + j + v]), wj, acc[r]);
      }
    }
  }
  // reduce each row's accumulator over the workgroup (wave sums, then 4 waves)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    W s = vconv<W>(acc[r]);
    s = wave_sum(s);
    if (lane == 0) red[r][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x < RB && threadIdx.x < rows) {
    const int r = threadIdx.x;
    W s = vadd(vadd(red[r][0], red[r][1]), vadd(red[r][2], red[r][3]));
    qpart[(int64_t)bk.x * m + i0 + r] = s;
  }
}
template <typename V, typename C, typename W, int RB, int VEC>
__global__ void __launch_bounds__(256) k_gemv_fwd(const V* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                  const C* __restrict__ w, int64_t chunk,
                                                  W* __restrict__ qpart, const int32_t* __restrict__ flag) {
  k_gemv_fwd_body<V, C, W, RB, VEC>(bk_hw(), A, lda, m, n, w, chunk, qpart, flag);
}

// ---------------------------------------------------------------------------
// Fused pass  q = A (A* p)  reading A once (m <= 32 * RPT).
// Workgroup g (TPB threads) streams column strips of width Wd = 8 * CPT (256
// bytes of each row).  Thread t owns columns cg*CPT .. +CPT-1 (cg = t % 8) of
// the strip and rows rg + (TPB/8) k, k < RPT (rg = t / 8), in registers, so
// 8 adjacent lanes read one contiguous 256-byte row segment.  Per strip:
//   t_c = sum_r conj(A_rc) p_r   (over rows: lane distances 8, 16, 32, then
//                                 the waves via LDS)
//   qacc_r += sum_c A_rc t_c     (registers, reduced over column groups once
//                                 per workgroup at the end)
// Output: qpart[g * m + i], FP64; the strips of a workgroup are contiguous.
// WT: also store every entry read into the column-major copy At (column c
// at At + c ldt); for one register slot the lanes of a wave then write 8
// columns x 8 consecutive rows, 128-byte runs.
template <typename V, typename C, typename U, int CPT, int RPT, int TPB, int VEC, bool WT = false>
__device__ __forceinline__ void k_gram_body(const Bk bk, const V* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                              const U* __restrict__ p, int64_t strips_per_wg, int64_t nstrips,
                                              U* __restrict__ qpart, const int32_t* __restrict__ flag,
                                              int interleave, V* __restrict__ At = nullptr, int64_t ldt = 0) {
  if (stopped(flag)) return;
  constexpr int WD = 8 * CPT;
  // VEC: elements per load (16 bytes when rows are 16-byte aligned, else 1)
  constexpr int LPR = CPT / VEC;    // loads per row segment
  constexpr int RG = TPB / 8;       // row groups
  constexpr int NW = TPB / 64;      // waves
  __shared__ C sp[RG * RPT];
  __shared__ C red[2][NW][WD];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int cg = t & 7, rg = t >> 3;
  for (int64_t i = t; i < RG * RPT; i += TPB) sp[i] = (i < m) ? vconv<C>(p[i]) : vzero<C>();
  C qacc[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) qacc[k] = vzero<C>();
  // this workgroup's strips: a contiguous run, or (interleave) every
  // bk.gx-th strip, so that the workgroups in flight read neighbouring
  // columns rather than addresses one run apart
  int64_t s0, s1, sstep;
  if (interleave) {
    s0 = bk.x;
    s1 = nstrips;
    sstep = bk.gx;
  } else {
    s0 = (int64_t)bk.x * strips_per_wg;
    s1 = s0 + strips_per_wg;
    if (s1 > nstrips) s1 = nstrips;
    sstep = 1;
  }
  __syncthreads();
  // strip loads into registers; two register sets so that the next strip's
  // loads are in flight while the current one is reduced
  auto load_strip = [&](V (&x)[RPT][CPT], int64_t sidx) {
    const int64_t cbase = sidx * WD + cg * CPT;
    const bool full = cbase + CPT <= n;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int64_t r = rg + RG * k;
      if (r < m && full) {
#pragma unroll
        for (int q = 0; q < LPR; ++q) {
          const Pack<V, VEC> pk = loadk<V, VEC>(A + r * lda + cbase + q * VEC);
#pragma unroll
          for (int v = 0; v < VEC; ++v) x[k][q * VEC + v] = pk.v[v];
        }
      } else {
#pragma unroll
        for (int u = 0; u < CPT; ++u) x[k][u] = (r < m && cbase + u < n) ? A[r * lda + cbase + u] : vzero<V>();
      }
      if constexpr (WT) {
#pragma unroll
        for (int u = 0; u < CPT; ++u)
          if (r < m && cbase + u < n) At[(cbase + u) * ldt + r] = x[k][u];
      }
    }
  };
  int slot = 0;
  auto process = [&](const V (&x)[RPT][CPT]) {
    C tp[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) tp[u] = vzero<C>();
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const C pr = sp[rg + RG * k];
#pragma unroll
      for (int u = 0; u < CPT; ++u) tp[u] = vcfma(vconv<C>(x[k][u]), pr, tp[u]);
    }
    // reduce over the 8 row groups of this wave (lanes equal mod 8): lane
    // distance 8 by a DPP rotation within 16-lane rows, then 16 and 32
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      tp[u] = vadd(tp[u], dpp<kDppRor8>(tp[u]));
      if constexpr (VT<C>::cplx) {
        tp[u].re += __shfl_xor(tp[u].re, 16, 64);
        tp[u].im += __shfl_xor(tp[u].im, 16, 64);
        tp[u].re += __shfl_xor(tp[u].re, 32, 64);
        tp[u].im += __shfl_xor(tp[u].im, 32, 64);
      } else {
        tp[u] += __shfl_xor(tp[u], 16, 64);
        tp[u] += __shfl_xor(tp[u], 32, 64);
      }
    }
    if (lane < 8) {
#pragma unroll
      for (int u = 0; u < CPT; ++u) red[slot][wv][lane * CPT + u] = tp[u];
    }
    __syncthreads();
    C tc[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int c = cg * CPT + u;
      C sum = red[slot][0][c];
#pragma unroll
      for (int w = 1; w < NW; ++w) sum = vadd(sum, red[slot][w][c]);
      tc[u] = sum;
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k)
#pragma unroll
      for (int u = 0; u < CPT; ++u) qacc[k] = vfma(vconv<C>(x[k][u]), tc[u], qacc[k]);
    slot ^= 1;
  };
  V xa[RPT][CPT], xb[RPT][CPT];
  if (s0 < s1) load_strip(xa, s0);
  for (int64_t sidx = s0; sidx < s1; sidx += 2 * sstep) {
    if (sidx + sstep < s1) load_strip(xb, sidx + sstep);
    process(xa);
    if (sidx + sstep < s1) {
      if (sidx + 2 * sstep < s1) load_strip(xa, sidx + 2 * sstep);
      process(xb);
    }
  }
  // reduce q over the 8 column groups (low 3 lane bits) and write this
  // workgroup's partial
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    U v = vconv<U>(qacc[k]);
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) {
      if constexpr (VT<U>::cplx) {
        v.re += __shfl_xor(v.re, off, 64);
        v.im += __shfl_xor(v.im, off, 64);
      } else {
        v += __shfl_xor(v, off, 64);
      }
    }
    const int64_t r = rg + RG * k;
    if (cg == 0 && r < m) qpart[(int64_t)bk.x * m + r] = v;
  }
}
template <typename V, typename C, typename U, int CPT, int RPT, int TPB, int VEC>
__global__ void __launch_bounds__(TPB) k_gram(const V* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                              const U* __restrict__ p, int64_t strips_per_wg, int64_t nstrips,
                                              U* __restrict__ qpart, const int32_t* __restrict__ flag,
                                              int interleave) {
  k_gram_body<V, C, U, CPT, RPT, TPB, VEC>(bk_hw(), A, lda, m, n, p, strips_per_wg, nstrips, qpart, flag, interleave);
}
// the same pass, also writing the column-major copy At
template <typename V, typename C, typename U, int CPT, int RPT, int TPB, int VEC>
__global__ void __launch_bounds__(TPB) k_gram_wt(const V* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                 const U* __restrict__ p, int64_t strips_per_wg, int64_t nstrips,
                                                 U* __restrict__ qpart, const int32_t* __restrict__ flag,
                                                 int interleave, V* __restrict__ At, int64_t ldt) {
  k_gram_body<V, C, U, CPT, RPT, TPB, VEC, true>(bk_hw(), A, lda, m, n, p, strips_per_wg, nstrips, qpart, flag,
                                                 interleave, At, ldt);
}

// ---------------------------------------------------------------------------
// Fused pass q = A (A* p) from the column-major copy At (column c of A at
// At + c ldt, its m rows contiguous), m <= 64 RPT.  512 threads; strips of
// 8 CPT columns, wave w takes columns w CPT .. w CPT + CPT - 1 of each strip
// and lane l rows l + 64 k (k < RPT) of them, so one load instruction of a
// wave reads 64 consecutive entries of one column and a wave streams CPT
// whole columns per strip.  The column sums t_c = sum_r conj(A_rc) p_r are a
// single all-lane wave reduction -- no LDS and no barrier per strip, the
// waves run decoupled -- and q_r += sum_c A_rc t_c stays in registers until
// one reduction over the 8 waves at the end.  Output as k_gram.
template <typename V, typename C, typename U, int CPT, int RPT>
__device__ __forceinline__ void k_gram_cm_body(const Bk bk, const V* __restrict__ At, int64_t ldt, int64_t m,
                                                 int64_t n, const U* __restrict__ p, int64_t strips_per_wg,
                                                 int64_t nstrips, U* __restrict__ qpart,
                                                 const int32_t* __restrict__ flag, int interleave) {
  if (stopped(flag)) return;
  constexpr int WD = 8 * CPT;
  __shared__ U red[8][64 * RPT];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int g = bk.x, G = bk.gx;
  C pr[RPT], qacc[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int64_t r = lane + 64 * k;
    pr[k] = r < m ? vconv<C>(p[r]) : vzero<C>();
    qacc[k] = vzero<C>();
  }
  int64_t s0, s1, sstep;
  if (interleave) {
    s0 = g;
    s1 = nstrips;
    sstep = G;
  } else {
    s0 = (int64_t)g * strips_per_wg;
    s1 = s0 + strips_per_wg;
    if (s1 > nstrips) s1 = nstrips;
    sstep = 1;
  }
  auto load_strip = [&](V (&x)[RPT][CPT], int64_t sidx) {
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int64_t c = sidx * WD + wv * CPT + u;
      const V* col = At + c * ldt;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int64_t r = lane + 64 * k;
        x[k][u] = (c < n && r < m) ? ld_once(col + r) : vzero<V>();
      }
    }
  };
  auto process = [&](const V (&x)[RPT][CPT]) {
    C tc[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      C a = vzero<C>();
#pragma unroll
      for (int k = 0; k < RPT; ++k) a = vcfma(vconv<C>(x[k][u]), pr[k], a);
      tc[u] = wave_sum(a);
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k)
#pragma unroll
      for (int u = 0; u < CPT; ++u) qacc[k] = vfma(vconv<C>(x[k][u]), tc[u], qacc[k]);
  };
  V xa[RPT][CPT], xb[RPT][CPT];
  if (s0 < s1) load_strip(xa, s0);
  for (int64_t sidx = s0; sidx < s1; sidx += 2 * sstep) {
    if (sidx + sstep < s1) load_strip(xb, sidx + sstep);
    process(xa);
    if (sidx + sstep < s1) {
      if (sidx + 2 * sstep < s1) load_strip(xa, sidx + 2 * sstep);
      process(xb);
    }
  }
  // sum over the 8 waves (fixed order) and write this workgroup's partial
#pragma unroll
  for (int k = 0; k < RPT; ++k) red[wv][lane + 64 * k] = vconv<U>(qacc[k]);
  __syncthreads();
  for (int r = t; r < 64 * RPT; r += 512) {
    U v = red[0][r];
#pragma unroll
    for (int w = 1; w < 8; ++w) v = vadd(v, red[w][r]);
    if (r < m) qpart[(int64_t)g * m + r] = v;
  }
}
template <typename V, typename C, typename U, int CPT, int RPT>
__global__ void __launch_bounds__(512) k_gram_cm(const V* __restrict__ At, int64_t ldt, int64_t m, int64_t n,
                                                 const U* __restrict__ p, int64_t strips_per_wg, int64_t nstrips,
                                                 U* __restrict__ qpart, const int32_t* __restrict__ flag,
                                                 int interleave) {
  k_gram_cm_body<V, C, U, CPT, RPT>(bk_hw(), At, ldt, m, n, p, strips_per_wg, nstrips, qpart, flag, interleave);
}

// ---------------------------------------------------------------------------
// The fused pass q = A (A* p) from the column-major copy for tall A (m up to
// WPC * 64 * RPT, beyond the 512 rows one wave holds in k_gram_cm).  A column
// group of WPC waves streams CPT whole columns per step: wave w of the group
// holds rows w 64 RPT .. (w + 1) 64 RPT - 1 of them, VPL consecutive rows per
// 16-byte load (lane l, load k: rows w 64 RPT + (64 k + l) VPL + v), so each
// load instruction of a wave reads 1 KB of one column.  The column sums
// t_c = sum_r conj(A_rc) p_r are a wave reduction per wave and, for WPC > 1,
// a sum of the WPC wave results through LDS in wave order (one barrier per
// step, two LDS slots so the next step's writes never meet this step's
// reads); then q_r += A_rc t_c in registers.  The next step's columns load
// into a second register set while the current one is reduced.  Column
// group gc of workgroup g takes columns (s (G NG) + g NG + gc) CPT + u at
// step s, so the grid's groups read neighbouring columns.  Rows m .. ldt - 1
// of the copy are zero, and every group runs the same number of steps (a
// column past n loads as zero), so the barriers are uniform.  At the end the
// NG groups' q are added in group order through LDS and each workgroup
// writes its partial as k_gram does.
template <typename V, typename C, typename U, int RPT, int CPT, int WPC, int TPB>
__device__ __forceinline__ void k_gram_tall_body(const Bk bk, const V* __restrict__ At, int64_t ldt, int64_t m,
                                                   int64_t n, const U* __restrict__ p, U* __restrict__ qpart,
                                                   const int32_t* __restrict__ flag) {
  if (stopped(flag)) return;
  constexpr int VPL = Vec16<V>::n;      // rows per 16-byte load
  constexpr int KL = RPT / VPL;         // loads per column and lane
  constexpr int NW = TPB / 64;          // waves
  constexpr int NG = NW / WPC;          // column groups
  constexpr int SLAB = 64 * RPT;        // rows per wave
  static_assert(RPT % VPL == 0 && NW % WPC == 0, "tall pass shape");
  __shared__ C red[2][NG][WPC][CPT];
  __shared__ U qs[WPC * SLAB];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int gc = wv / WPC, w = wv % WPC;
  const int64_t r0 = (int64_t)w * SLAB;
  // loads of this wave that fall inside the copy's ldt rows (uniform)
  int64_t kl = (ldt - r0) / (64 * VPL);
  const int kmax = kl < 0 ? 0 : (kl > KL ? KL : (int)kl);
  C pr[KL][VPL], qacc[KL][VPL];
#pragma unroll
  for (int k = 0; k < KL; ++k)
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
      const int64_t r = r0 + (64 * k + lane) * VPL + v;
      pr[k][v] = r < m ? vconv<C>(p[r]) : vzero<C>();
      qacc[k][v] = vzero<C>();
    }
  const int64_t groups = (int64_t)bk.gx * NG;
  const int64_t gid = (int64_t)bk.x * NG + gc;
  const int64_t steps = ceil_div(n, groups * CPT);
  auto load = [&](Pack<V, VPL> (&x)[KL][CPT], int64_t s) {
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int64_t c = (s * groups + gid) * CPT + u;
      const V* col = At + c * ldt + r0 + (int64_t)lane * VPL;
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        if (c < n && k < kmax) x[k][u] = loadk_once<V, VPL>(col + 64 * VPL * k);
        else
#pragma unroll
          for (int v = 0; v < VPL; ++v) x[k][u].v[v] = vzero<V>();
      }
    }
  };
  int slot = 0;
  auto process = [&](const Pack<V, VPL> (&x)[KL][CPT]) {
    C tc[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      C a = vzero<C>();
#pragma unroll
      for (int k = 0; k < KL; ++k)
#pragma unroll
        for (int v = 0; v < VPL; ++v) a = vcfma(vconv<C>(x[k][u].v[v]), pr[k][v], a);
      tc[u] = wave_sum(a);
    }
    if constexpr (WPC > 1) {
      if (lane == 0)
#pragma unroll
        for (int u = 0; u < CPT; ++u) red[slot][gc][w][u] = tc[u];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        C s = red[slot][gc][0][u];
#pragma unroll
        for (int ww = 1; ww < WPC; ++ww) s = vadd(s, red[slot][gc][ww][u]);
        tc[u] = s;
      }
      slot ^= 1;
    }
#pragma unroll
    for (int k = 0; k < KL; ++k)
#pragma unroll
      for (int v = 0; v < VPL; ++v)
#pragma unroll
        for (int u = 0; u < CPT; ++u) qacc[k][v] = vfma(vconv<C>(x[k][u].v[v]), tc[u], qacc[k][v]);
  };
  Pack<V, VPL> xa[KL][CPT], xb[KL][CPT];
  if (steps > 0) load(xa, 0);
  for (int64_t s = 0; s < steps; s += 2) {
    if (s + 1 < steps) load(xb, s + 1);
    process(xa);
    if (s + 1 < steps) {
      if (s + 2 < steps) load(xa, s + 2);
      process(xb);
    }
  }
  // the NG groups' q, added in group order, then this workgroup's partial
  for (int g2 = 0; g2 < NG; ++g2) {
    __syncthreads();
    if (gc == g2)
#pragma unroll
      for (int k = 0; k < KL; ++k)
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
          const int i = w * SLAB + (64 * k + lane) * VPL + v;
          const U val = vconv<U>(qacc[k][v]);
          qs[i] = g2 == 0 ? val : vadd(qs[i], val);
        }
  }
  __syncthreads();
  for (int64_t r = t; r < m; r += TPB) qpart[(int64_t)bk.x * m + r] = qs[r];
}
template <typename V, typename C, typename U, int RPT, int CPT, int WPC, int TPB>
__global__ void __launch_bounds__(TPB) k_gram_tall(const V* __restrict__ At, int64_t ldt, int64_t m, int64_t n,
                                                   const U* __restrict__ p, U* __restrict__ qpart,
                                                   const int32_t* __restrict__ flag) {
  k_gram_tall_body<V, C, U, RPT, CPT, WPC, TPB>(bk_hw(), At, ldt, m, n, p, qpart, flag);
}

// Column-major copy of a row-major m x n matrix: At[c ldt + r] = A[r lda + c]
// for r < m, zero for m <= r < ldt.  Tiles of 64 rows x TW columns (1 KB of a
// row: TW = 64 complex128 or 128 complex64 entries) through LDS (one padding
// column against bank conflicts); rows are read and columns written as
// contiguous 1 KB and 512-1024 B runs by consecutive threads, and each thread
// issues all its loads of a tile before storing any.  grid (ceil(n / TW),
// ldt / 64), 256 threads.
template <typename V>
__device__ __forceinline__ void colmajor_tile(int bx, int by, const V* __restrict__ A, int64_t lda, int64_t m,
                                              int64_t n, V* __restrict__ At, int64_t ldt) {
  constexpr int TW = 1024 / (int)sizeof(V) < 64 ? 1024 / (int)sizeof(V) : (1024 / (int)sizeof(V) > 128 ? 128 : 1024 / (int)sizeof(V));
  constexpr int PER = 64 * TW / 256;  // entries per thread
  __shared__ V tile[64][TW + 1];
  const int64_t c0 = (int64_t)bx * TW, r0 = (int64_t)by * 64;
  const int tid = threadIdx.x;
  V v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 256 * u, rr = e / TW, cc = e % TW;
    const int64_t r = r0 + rr, c = c0 + cc;
    v[u] = (r < m && c < n) ? ld_once(A + r * lda + c) : vzero<V>();
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 256 * u;
    tile[e / TW][e % TW] = v[u];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 256 * u, cc = e / 64, rr = e % 64;
    v[u] = tile[rr][cc];
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 256 * u, cc = e / 64, rr = e % 64;
    const int64_t c = c0 + cc;
    if (c < n) At[c * ldt + r0 + rr] = v[u];
  }
}
template <typename V>
__global__ void __launch_bounds__(256) k_colmajor(const V* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                  V* __restrict__ At, int64_t ldt) {
  colmajor_tile<V>((int)blockIdx.x, (int)blockIdx.y, A, lda, m, n, At, ldt);
}
template <typename V> constexpr int colmajor_tw() {
  return 1024 / (int)sizeof(V) < 64 ? 1024 / (int)sizeof(V) : (1024 / (int)sizeof(V) > 128 ? 128 : 1024 / (int)sizeof(V));
}
// every system's column-major copy At of its bulk matrix Ab (batched form):
// the system's grid is (ceil(n / TW), ldt / 64) tiles
template <typename V>
__global__ void __launch_bounds__(256) kb_colmajor(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                   int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  const Bk bk = bgrid_local(grid[i], (int)blockIdx.x - grid[i].start);
  colmajor_tile<V>(bk.x, bk.y, reinterpret_cast<const V*>(s.Ab), s.ldab, s.m, s.n, reinterpret_cast<V*>(s.At),
                   s.ldt);
}

// q[i] = sum over the pass's G workgroup partials qpart[g * m + i], in a
// fixed order: 16 rows per workgroup, the 16 lane groups of a row each take
// every sixteenth g, then the group sums are added in group order.
// grid = ceil(m / 16), 256 threads.
template <typename U>
__device__ __forceinline__ void k_gram_reduce_body(const Bk bk, const U* __restrict__ qpart, int G, int64_t m,
                                                     U* __restrict__ q, const int32_t* __restrict__ flag) {
  if (stopped(flag)) return;
  __shared__ U red[16][16];
  const int rr = threadIdx.x & 15, part = threadIdx.x >> 4;
  const int64_t i = (int64_t)bk.x * 16 + rr;
  U a0 = vzero<U>(), a1 = vzero<U>();
  if (i < m) {
    int g = part;
    for (; g + 16 < G; g += 32) {
      a0 = vadd(a0, qpart[(int64_t)g * m + i]);
      a1 = vadd(a1, qpart[(int64_t)(g + 16) * m + i]);
    }
    if (g < G) a0 = vadd(a0, qpart[(int64_t)g * m + i]);
  }
  red[part][rr] = vadd(a0, a1);
  __syncthreads();
  if (part == 0 && i < m) {
    U t = red[0][rr];
#pragma unroll
    for (int k = 1; k < 16; ++k) t = vadd(t, red[k][rr]);
    q[i] = t;
  }
}
template <typename U>
__global__ void __launch_bounds__(256) k_gram_reduce(const U* __restrict__ qpart, int G, int64_t m,
                                                     U* __restrict__ q, const int32_t* __restrict__ flag) {
  k_gram_reduce_body<U>(bk_hw(), qpart, G, m, q, flag);
}

// ---------------------------------------------------------------------------
__host__ __device__ static inline bool aligned16(const void* p, int64_t ld, int64_t es) {
  return ((uintptr_t)p % 16 == 0) && ((ld * es) % 16 == 0);
}

static int64_t slabs_for(int64_t m, int64_t n, int vec) {
  const int64_t nb = ceil_div(n, (int64_t)256 * vec);
  // enough workgroups to fill the chip (~2048), slabs of at least 32 rows
  int64_t rs = ceil_div(2048, nb);
  if (rs > ceil_div(m, 32)) rs = ceil_div(m, 32);
  if (rs < 1) rs = 1;
  if (rs > kMaxSlabs) rs = kMaxSlabs;
  const int64_t rps = ceil_div(m, rs);
  return ceil_div(m, rps);
}

template <typename V, typename C, typename W, int VEC>
static hipError_t adj_run(const AdjArgs& a, hipStream_t st) {
  const int64_t nb = ceil_div(a.n, (int64_t)256 * VEC);
  int64_t rs = slabs_for(a.m, a.n, VEC);
  const int64_t rps = ceil_div(a.m, rs);
  const V* A = reinterpret_cast<const V*>(a.A);
  const W* u = reinterpret_cast<const W*>(a.u);
  C* w = reinterpret_cast<C*>(a.w);
  W* wide = reinterpret_cast<W*>(a.w_wide);
  // the timing events (if any) belong to the dispatch itself
  if (rs == 1 && wide == nullptr) {
    hipExtLaunchKernelGGL((k_gemv_adj<V, C, W, VEC>), dim3((unsigned)nb, 1), dim3(256), 0, st, a.ev_begin, a.ev_end,
                          0, A, a.lda, a.m, a.n, u, rps, w, a.flag);
    return hipGetLastError();
  }
  C* part = reinterpret_cast<C*>(a.part);
  hipExtLaunchKernelGGL((k_gemv_adj<V, C, W, VEC>), dim3((unsigned)nb, (unsigned)rs), dim3(256), 0, st, a.ev_begin,
                        a.ev_end, 0, A, a.lda, a.m, a.n, u, rps, part, a.flag);
  hipLaunchKernelGGL((k_sum_slabs<C, W>), dim3((unsigned)ceil_div(a.n, 256)), dim3(256), 0, st, part, (int)rs, a.n,
                     w, wide, a.flag);
  return hipGetLastError();
}

template <typename V, typename C, typename W>
static hipError_t adj_impl(const AdjArgs& a, hipStream_t st) {
  if (aligned16(a.A, a.lda, sizeof(V))) return adj_run<V, C, W, Vec16<V>::n>(a, st);
  return adj_run<V, C, W, 1>(a, st);
}

template <typename V, typename C, typename W, int VEC>
static hipError_t fwd_run(const FwdArgs& a, hipStream_t st) {
  constexpr int RB = 8;
  const int64_t rb = ceil_div(a.m, RB);
  int64_t cs = ceil_div(2048, rb);
  const int64_t min_chunk = 256 * VEC * 2;
  if (cs > ceil_div(a.n, min_chunk)) cs = ceil_div(a.n, min_chunk);
  if (cs < 1) cs = 1;
  if (cs > kMaxChunks) cs = kMaxChunks;
  int64_t chunk = ceil_div(a.n, cs);
  chunk = ceil_div(chunk, 256 * VEC) * (256 * VEC);
  cs = ceil_div(a.n, chunk);
  hipExtLaunchKernelGGL((k_gemv_fwd<V, C, W, RB, VEC>), dim3((unsigned)cs, (unsigned)rb), dim3(256), 0, st,
                        a.ev_begin, a.ev_end, 0, reinterpret_cast<const V*>(a.A), a.lda, a.m, a.n,
                        reinterpret_cast<const C*>(a.w), chunk, reinterpret_cast<W*>(a.qpart), a.flag);
  if (a.chunks_out) *a.chunks_out = (int)cs;
  return hipGetLastError();
}

template <typename V, typename C, typename W>
static hipError_t fwd_impl(const FwdArgs& a, hipStream_t st) {
  if (aligned16(a.A, a.lda, sizeof(V))) return fwd_run<V, C, W, Vec16<V>::n>(a, st);
  return fwd_run<V, C, W, 1>(a, st);
}

// the widest vector (4 elements) gives the fewest column blocks and hence
// the most slabs: size the partial buffer for that case
template <typename V, typename C, typename U, int CPT, int VEC>
static hipError_t gram_go(const GramArgs& a, hipStream_t st) {
  constexpr int WD = 8 * CPT;
  const int64_t nstrips = ceil_div(a.n, WD);
  const int64_t maxwg = a.max_wg > 0 && a.max_wg <= kGramMaxWg ? a.max_wg : 512;
  int64_t G = nstrips < maxwg ? nstrips : maxwg;
  const int64_t spw = ceil_div(nstrips, G);
  G = ceil_div(nstrips, spw);
  const V* A = reinterpret_cast<const V*>(a.A);
  const U* p = reinterpret_cast<const U*>(a.p);
  U* qpart = reinterpret_cast<U*>(a.qpart);
  if (a.at_mode == 1) {
    // the pass that also writes the column-major copy (512 threads)
    V* At = reinterpret_cast<V*>(a.At);
    if (a.m <= 64)
      hipLaunchKernelGGL((k_gram_wt<V, C, U, CPT, 1, 512, VEC>), dim3((unsigned)G), dim3(512), 0, st, A, a.lda, a.m,
                         a.n, p, spw, nstrips, qpart, a.flag, a.interleave, At, a.ldt);
    else if (a.m <= 128)
      hipLaunchKernelGGL((k_gram_wt<V, C, U, CPT, 2, 512, VEC>), dim3((unsigned)G), dim3(512), 0, st, A, a.lda, a.m,
                         a.n, p, spw, nstrips, qpart, a.flag, a.interleave, At, a.ldt);
    else if (a.m <= 256)
      hipLaunchKernelGGL((k_gram_wt<V, C, U, CPT, 4, 512, VEC>), dim3((unsigned)G), dim3(512), 0, st, A, a.lda, a.m,
                         a.n, p, spw, nstrips, qpart, a.flag, a.interleave, At, a.ldt);
    else
      hipLaunchKernelGGL((k_gram_wt<V, C, U, CPT, 8, 512, VEC>), dim3((unsigned)G), dim3(512), 0, st, A, a.lda, a.m,
                         a.n, p, spw, nstrips, qpart, a.flag, a.interleave, At, a.ldt);
  } else if (a.wide_wg) {
    // 1024 threads: 128 row groups, RPT rows each
    if (a.m <= 128)
      hipExtLaunchKernelGGL((k_gram<V, C, U, CPT, 1, 1024, VEC>), dim3((unsigned)G), dim3(1024), 0, st, a.ev_begin,
                            a.ev_end, 0, A, a.lda, a.m, a.n, p, spw, nstrips, qpart, a.flag, a.interleave);
    else if (a.m <= 256)
      hipExtLaunchKernelGGL((k_gram<V, C, U, CPT, 2, 1024, VEC>), dim3((unsigned)G), dim3(1024), 0, st, a.ev_begin,
                            a.ev_end, 0, A, a.lda, a.m, a.n, p, spw, nstrips, qpart, a.flag, a.interleave);
    else
      hipExtLaunchKernelGGL((k_gram<V, C, U, CPT, 4, 1024, VEC>), dim3((unsigned)G), dim3(1024), 0, st, a.ev_begin,
                            a.ev_end, 0, A, a.lda, a.m, a.n, p, spw, nstrips, qpart, a.flag, a.interleave);
  } else if (a.m <= 64) {
    // 512 threads: 64 row groups, RPT rows each
    hipExtLaunchKernelGGL((k_gram<V, C, U, CPT, 1, 512, VEC>), dim3((unsigned)G), dim3(512), 0, st, a.ev_begin,
                          a.ev_end, 0, A, a.lda, a.m, a.n, p, spw, nstrips, qpart, a.flag, a.interleave);
  } else if (a.m <= 128) {
    hipExtLaunchKernelGGL((k_gram<V, C, U, CPT, 2, 512, VEC>), dim3((unsigned)G), dim3(512), 0, st, a.ev_begin,
                          a.ev_end, 0, A, a.lda, a.m, a.n, p, spw, nstrips, qpart, a.flag, a.interleave);
  } else if (a.m <= 256) {
    hipExtLaunchKernelGGL((k_gram<V, C, U, CPT, 4, 512, VEC>), dim3((unsigned)G), dim3(512), 0, st, a.ev_begin,
                          a.ev_end, 0, A, a.lda, a.m, a.n, p, spw, nstrips, qpart, a.flag, a.interleave);
  } else {
    hipExtLaunchKernelGGL((k_gram<V, C, U, CPT, 8, 512, VEC>), dim3((unsigned)G), dim3(512), 0, st, a.ev_begin,
                          a.ev_end, 0, A, a.lda, a.m, a.n, p, spw, nstrips, qpart, a.flag, a.interleave);
  }
  hipLaunchKernelGGL((k_gram_reduce<U>), dim3((unsigned)ceil_div(a.m, 16)), dim3(256), 0, st, qpart, (int)G,
                     a.m, reinterpret_cast<U*>(a.q), a.flag);
  return hipGetLastError();
}

// The pass over the column-major copy: RPT = ceil(m / 64) rows per lane
// (1, 2, 4, 8) and CPT = 16 / RPT columns per wave and strip, at most 8
// (16 entries per lane and register set, 8 for m <= 64).
template <typename V, typename C, typename U>
static hipError_t gram_cm_go(const GramArgs& a, hipStream_t st) {
  const int rpt = a.m <= 64 ? 1 : (a.m <= 128 ? 2 : (a.m <= 256 ? 4 : 8));
  const int64_t WD = 8 * (rpt == 1 ? 8 : 16 / rpt);
  const int64_t nstrips = ceil_div(a.n, WD);
  const int64_t maxwg = a.max_wg > 0 && a.max_wg <= kGramMaxWg ? a.max_wg : 512;
  int64_t G = nstrips < maxwg ? nstrips : maxwg;
  const int64_t spw = ceil_div(nstrips, G);
  G = ceil_div(nstrips, spw);
  const V* At = reinterpret_cast<const V*>(a.At);
  const U* p = reinterpret_cast<const U*>(a.p);
  U* qpart = reinterpret_cast<U*>(a.qpart);
  if (rpt == 1)
    hipExtLaunchKernelGGL((k_gram_cm<V, C, U, 8, 1>), dim3((unsigned)G), dim3(512), 0, st, a.ev_begin, a.ev_end, 0,
                          At, a.ldt, a.m, a.n, p, spw, nstrips, qpart, a.flag, a.interleave);
  else if (rpt == 2)
    hipExtLaunchKernelGGL((k_gram_cm<V, C, U, 8, 2>), dim3((unsigned)G), dim3(512), 0, st, a.ev_begin, a.ev_end, 0,
                          At, a.ldt, a.m, a.n, p, spw, nstrips, qpart, a.flag, a.interleave);
  else if (rpt == 4)
    hipExtLaunchKernelGGL((k_gram_cm<V, C, U, 4, 4>), dim3((unsigned)G), dim3(512), 0, st, a.ev_begin, a.ev_end, 0,
                          At, a.ldt, a.m, a.n, p, spw, nstrips, qpart, a.flag, a.interleave);
  else
    hipExtLaunchKernelGGL((k_gram_cm<V, C, U, 2, 8>), dim3((unsigned)G), dim3(512), 0, st, a.ev_begin, a.ev_end, 0,
                          At, a.ldt, a.m, a.n, p, spw, nstrips, qpart, a.flag, a.interleave);
  hipLaunchKernelGGL((k_gram_reduce<U>), dim3((unsigned)ceil_div(a.m, 16)), dim3(256), 0, st, qpart, (int)G,
                     a.m, reinterpret_cast<U*>(a.q), a.flag);
  return hipGetLastError();
}

// The tall pass (m > kGramMaxRows): shape code a.tall (RPT, CPT, WPC, TPB
// below) for the row class m <= 1024 or m <= 2048; at_mode 1 first writes the
// column-major copy (k_colmajor), then runs the pass over it.
template <typename V, typename C, typename U, int RPT, int CPT, int WPC, int TPB>
static void tall_launch(const GramArgs& a, int64_t G, hipStream_t st) {
  hipExtLaunchKernelGGL((k_gram_tall<V, C, U, RPT, CPT, WPC, TPB>), dim3((unsigned)G), dim3(TPB), 0, st, a.ev_begin,
                        a.ev_end, 0, reinterpret_cast<const V*>(a.At), a.ldt, a.m, a.n,
                        reinterpret_cast<const U*>(a.p), reinterpret_cast<U*>(a.qpart), a.flag);
}
template <typename V, typename C, typename U>
static hipError_t gram_tall_go(const GramArgs& a, hipStream_t st) {
  if (a.m > kGramTallMaxRows || a.ldt < a.m || a.ldt % gram_tall_ld_multiple() != 0) return hipErrorInvalidValue;
  if (a.at_mode == 1) {
    hipLaunchKernelGGL((k_colmajor<V>), dim3((unsigned)ceil_div(a.n, colmajor_tw<V>()), (unsigned)(a.ldt / 64)),
                       dim3(256), 0, st, reinterpret_cast<const V*>(a.A), a.lda, a.m, a.n, reinterpret_cast<V*>(a.At),
                       a.ldt);
  }
  const int64_t G = a.max_wg > 0 && a.max_wg <= kGramMaxWg ? a.max_wg : 512;
  const int code = a.tall & 3;
  if (a.m <= 1024) {
    switch (code) {
      case 0: tall_launch<V, C, U, 8, 2, 2, 256>(a, G, st); break;
      case 1: tall_launch<V, C, U, 4, 4, 4, 256>(a, G, st); break;
      case 2: tall_launch<V, C, U, 8, 1, 2, 256>(a, G, st); break;
      default: tall_launch<V, C, U, 16, 1, 1, 256>(a, G, st); break;
    }
  } else {
    switch (code) {
      case 0: tall_launch<V, C, U, 8, 2, 4, 256>(a, G, st); break;
      case 1: tall_launch<V, C, U, 4, 4, 8, 512>(a, G, st); break;
      case 2: tall_launch<V, C, U, 8, 1, 4, 256>(a, G, st); break;
      default: tall_launch<V, C, U, 16, 1, 2, 256>(a, G, st); break;
    }
  }
  hipLaunchKernelGGL((k_gram_reduce<U>), dim3((unsigned)ceil_div(a.m, 16)), dim3(256), 0, st,
                     reinterpret_cast<const U*>(a.qpart), (int)G, a.m, reinterpret_cast<U*>(a.q), a.flag);
  return hipGetLastError();
}

// Strip width: 32 bytes of a row per thread (CPT0), or half of that.
template <typename V, typename C, typename U>
static hipError_t gram_impl(const GramArgs& a, hipStream_t st) {
  if (a.m > kGramMaxRows) return gram_tall_go<V, C, U>(a, st);
  if (a.at_mode == 2) return gram_cm_go<V, C, U>(a, st);
  constexpr int CPT0 = 32 / (int)sizeof(V) > 0 ? 32 / (int)sizeof(V) : 1;
  constexpr int CPT1 = CPT0 / 2 > 0 ? CPT0 / 2 : 1;
  constexpr int VA = Vec16<V>::n;
  if (aligned16(a.A, a.lda, sizeof(V)))
    return a.narrow ? gram_go<V, C, U, CPT1, (CPT1 < VA ? CPT1 : VA)>(a, st) : gram_go<V, C, U, CPT0, VA>(a, st);
  return a.narrow ? gram_go<V, C, U, CPT1, 1>(a, st) : gram_go<V, C, U, CPT0, 1>(a, st);
}

bool gram_supported(int dtype, int64_t m, const void* A, int64_t lda) {
  (void)dtype;
  (void)A;
  (void)lda;
  return m <= kGramMaxRows;
}

int64_t gram_tall_ld_multiple() { return 256; }

int b_colmajor_tw(int dtype) {
  switch (dtype) {
    case 0: return colmajor_tw<cd>();
    case 1: return colmajor_tw<cf>();
    case 2: return colmajor_tw<double>();
    case 3: return colmajor_tw<float>();
  }
  return 0;
}

hipError_t launch_b_colmajor(int dtype, const BLaunch& L, hipStream_t st) {
  if (L.total <= 0) return hipSuccess;
  const dim3 grid((unsigned)L.total);
  switch (dtype) {
    case 0: hipLaunchKernelGGL((kb_colmajor<cd>), grid, dim3(256), 0, st, L.sys, L.grid, L.nsys); break;
    case 1: hipLaunchKernelGGL((kb_colmajor<cf>), grid, dim3(256), 0, st, L.sys, L.grid, L.nsys); break;
    case 2: hipLaunchKernelGGL((kb_colmajor<double>), grid, dim3(256), 0, st, L.sys, L.grid, L.nsys); break;
    case 3: hipLaunchKernelGGL((kb_colmajor<float>), grid, dim3(256), 0, st, L.sys, L.grid, L.nsys); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_colmajor(int dtype, const void* A, int64_t lda, int64_t m, int64_t n, void* At, int64_t ldt,
                           hipStream_t st) {
  if (ldt < m || ldt % 64 != 0) return hipErrorInvalidValue;
  const unsigned gy = (unsigned)(ldt / 64);
  switch (dtype) {
    case 0: hipLaunchKernelGGL((k_colmajor<cd>), dim3((unsigned)ceil_div(n, colmajor_tw<cd>()), gy), dim3(256), 0, st,
                               (const cd*)A, lda, m, n, (cd*)At, ldt); break;
    case 1: hipLaunchKernelGGL((k_colmajor<cf>), dim3((unsigned)ceil_div(n, colmajor_tw<cf>()), gy), dim3(256), 0, st,
                               (const cf*)A, lda, m, n, (cf*)At, ldt); break;
    case 2: hipLaunchKernelGGL((k_colmajor<double>), dim3((unsigned)ceil_div(n, colmajor_tw<double>()), gy), dim3(256),
                               0, st, (const double*)A, lda, m, n, (double*)At, ldt); break;
    case 3: hipLaunchKernelGGL((k_colmajor<float>), dim3((unsigned)ceil_div(n, colmajor_tw<float>()), gy), dim3(256),
                               0, st, (const float*)A, lda, m, n, (float*)At, ldt); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gram(int dtype, const GramArgs& a, hipStream_t st) {
  switch (dtype) {
    case 0: return gram_impl<cd, cd, cd>(a, st);
    case 1: return a.wide_acc ? gram_impl<cf, cd, cd>(a, st) : gram_impl<cf, cf, cd>(a, st);
    case 2: return gram_impl<double, double, double>(a, st);
    case 3: return a.wide_acc ? gram_impl<float, double, double>(a, st) : gram_impl<float, float, double>(a, st);
  }
  return hipErrorInvalidValue;
}

int64_t adj_part_elems(int64_t m, int64_t n) { return slabs_for(m, n, 4) * n; }

// dtype: storage of A; wide: accumulate in FP64 (w in FP64) even for
// single-precision storage.
hipError_t launch_gemv_adj(int dtype, bool wide, const AdjArgs& a, hipStream_t st) {
  switch (dtype) {
    case 0: return adj_impl<cd, cd, cd>(a, st);
    case 1: return wide ? adj_impl<cf, cd, cd>(a, st) : adj_impl<cf, cf, cd>(a, st);
    case 2: return adj_impl<double, double, double>(a, st);
    case 3: return wide ? adj_impl<float, double, double>(a, st) : adj_impl<float, float, double>(a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemv_fwd(int dtype, bool wide, const FwdArgs& a, hipStream_t st) {
  switch (dtype) {
    case 0: return fwd_impl<cd, cd, cd>(a, st);
    case 1: return wide ? fwd_impl<cf, cd, cd>(a, st) : fwd_impl<cf, cf, cd>(a, st);
    case 2: return fwd_impl<double, double, double>(a, st);
    case 3: return wide ? fwd_impl<float, double, double>(a, st) : fwd_impl<float, float, double>(a, st);
  }
  return hipErrorInvalidValue;
}

// ------------------------------ batched systems -------------------------------
namespace {

template <typename V, typename C, typename U, int CPT, int RPT, int VEC>
__global__ void __launch_bounds__(512) kb_gram(const BSys* __restrict__ sys, const BGrid* __restrict__ grid, int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_gram_body<V, C, U, CPT, RPT, 512, VEC>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start),
                                         reinterpret_cast<const V*>(s.Ab), s.ldab, s.m, s.n,
                                         reinterpret_cast<const U*>(s.p), s.gram_spw, s.gram_nstrips,
                                         reinterpret_cast<U*>(s.qpart), &s.st->done, 0);
}

// the same pass, also writing each system's column-major copy At (16-byte
// loads where the system's rows allow them); never skipped by the stop flag,
// so every copy is whole before a pass reads it
template <typename V, typename C, typename U, int CPT, int RPT, int VEC>
__global__ void __launch_bounds__(512) kb_gram_wt(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                  int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  const Bk bk = bgrid_local(grid[i], (int)blockIdx.x - grid[i].start);
  const V* A = reinterpret_cast<const V*>(s.Ab);
  if (aligned16(A, s.ldab, sizeof(V)))
    k_gram_body<V, C, U, CPT, RPT, 512, VEC, true>(bk, A, s.ldab, s.m, s.n, reinterpret_cast<const U*>(s.p),
                                                   s.gram_spw, s.gram_nstrips, reinterpret_cast<U*>(s.qpart),
                                                   nullptr, 0, reinterpret_cast<V*>(s.At), s.ldt);
  else
    k_gram_body<V, C, U, CPT, RPT, 512, 1, true>(bk, A, s.ldab, s.m, s.n, reinterpret_cast<const U*>(s.p),
                                                 s.gram_spw, s.gram_nstrips, reinterpret_cast<U*>(s.qpart), nullptr,
                                                 0, reinterpret_cast<V*>(s.At), s.ldt);
}

// the pass over each system's column-major copy
template <typename V, typename C, typename U, int CPT, int RPT>
__global__ void __launch_bounds__(512) kb_gram_cm(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                  int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_gram_cm_body<V, C, U, CPT, RPT>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start),
                                    reinterpret_cast<const V*>(s.At), s.ldt, s.m, s.n,
                                    reinterpret_cast<const U*>(s.p), s.cm_spw, s.cm_nstrips,
                                    reinterpret_cast<U*>(s.qpart), &s.st->done, 0);
}

template <typename U>
__global__ void __launch_bounds__(256) kb_gram_reduce(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                      int nsys, int use_flag) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_gram_reduce_body<U>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<const U*>(s.qpart),
                        s.gram_G, s.m, reinterpret_cast<U*>(s.q), use_flag ? &s.st->done : nullptr);
}

// FP64 residual product of the refinement, q = A (A* y_outer), as one fused
// pass over each system's problem data A (16-byte loads where its rows
// allow them); never skipped (the inner iteration's stop flag is set when a
// residual is due)
template <typename V, typename U, int CPT, int RPT>
__global__ void __launch_bounds__(512) kb_gram_res(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                   int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  const Bk bk = bgrid_local(grid[i], (int)blockIdx.x - grid[i].start);
  const V* A = reinterpret_cast<const V*>(s.A);
  if (aligned16(A, s.lda, sizeof(V)))
    k_gram_body<V, U, U, CPT, RPT, 512, Vec16<V>::n>(bk, A, s.lda, s.m, s.n, reinterpret_cast<const U*>(s.y_outer),
                                                     s.res_spw, s.res_nstrips, reinterpret_cast<U*>(s.qpart),
                                                     nullptr, 0);
  else
    k_gram_body<V, U, U, CPT, RPT, 512, 1>(bk, A, s.lda, s.m, s.n, reinterpret_cast<const U*>(s.y_outer), s.res_spw,
                                           s.res_nstrips, reinterpret_cast<U*>(s.qpart), nullptr, 0);
}

// A* u in FP64 into slab partials; u = y (use_y) or y_outer
template <typename V, typename W, int VEC>
__global__ void __launch_bounds__(256) kb_adj(const BSys* __restrict__ sys, const BGrid* __restrict__ grid, int nsys,
                                              int use_y) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_gemv_adj_body<V, W, W, VEC>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start),
                                reinterpret_cast<const V*>(s.A), s.lda, s.m, s.n,
                                reinterpret_cast<const W*>(use_y ? s.y : s.y_outer), s.adj_rps,
                                reinterpret_cast<W*>(s.apart), nullptr);
}

template <typename W>
__global__ void __launch_bounds__(256) kb_sum_slabs(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                    int nsys, int to_x) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_sum_slabs_body<W, W>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<const W*>(s.apart),
                         s.adj_slabs, s.n, reinterpret_cast<W*>(to_x ? s.x : s.w64), nullptr, nullptr);
}

template <typename V, typename W, int VEC>
__global__ void __launch_bounds__(256) kb_fwd(const BSys* __restrict__ sys, const BGrid* __restrict__ grid, int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_gemv_fwd_body<V, W, W, 8, VEC>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start),
                                   reinterpret_cast<const V*>(s.A), s.lda, s.m, s.n,
                                   reinterpret_cast<const W*>(s.w64), s.fwd_chunk, reinterpret_cast<W*>(s.fpart),
                                   nullptr);
}

template <typename V> int plan_gram_t(BSys& s, BGrid& gram, BGrid& red) {
  constexpr int CPT = 32 / (int)sizeof(V) > 0 ? 32 / (int)sizeof(V) : 1;
  const int64_t nstrips = ceil_div(s.n, 8 * CPT);
  // about 256 KB of A per workgroup (small systems take few workgroups)
  int64_t G = ceil_div(s.m * s.n * (int64_t)sizeof(V), 256 << 10);
  if (G > 512) G = 512;
  if (G > nstrips) G = nstrips;
  if (G < 1) G = 1;
  const int64_t spw = ceil_div(nstrips, G);
  G = ceil_div(nstrips, spw);
  s.gram_spw = spw;
  s.gram_nstrips = nstrips;
  s.gram_G = (int)G;
  // the pass over the column-major copy: the same G, its own strips (8 CPT'
  // columns, CPT' = 16 / rows per lane, at most 8)
  {
    const int rpt = s.m <= 64 ? 1 : (s.m <= 128 ? 2 : (s.m <= 256 ? 4 : 8));
    const int64_t wd = 8 * (rpt == 1 ? 8 : 16 / rpt);
    s.cm_nstrips = ceil_div(s.n, wd);
    s.cm_spw = ceil_div(s.cm_nstrips, G);
  }
  gram = BGrid{0, (int)G, 1, 1};
  red = BGrid{0, (int)ceil_div(s.m, 16), 1, 1};
  // rows per thread class: 512 threads hold 64 RPT rows
  return s.m <= 64 ? 0 : s.m <= 128 ? 1 : s.m <= 256 ? 2 : 3;
}

template <typename V> void plan_wide_t(bool aligned, BSys& s, BGrid& adj, BGrid& sum, BGrid& fwd) {
  const int VEC = aligned ? Vec16<V>::n : 1;
  const int64_t nb = ceil_div(s.n, (int64_t)256 * VEC);
  const int64_t rs = slabs_for(s.m, s.n, VEC);
  s.adj_slabs = (int)rs;
  s.adj_rps = ceil_div(s.m, rs);
  adj = BGrid{0, (int)nb, (int)rs, 1};
  sum = BGrid{0, (int)ceil_div(s.n, 256), 1, 1};
  const int64_t rb = ceil_div(s.m, 8);
  int64_t cs = ceil_div(2048, rb);
  const int64_t min_chunk = 256 * VEC * 2;
  if (cs > ceil_div(s.n, min_chunk)) cs = ceil_div(s.n, min_chunk);
  if (cs < 1) cs = 1;
  if (cs > kMaxChunks) cs = kMaxChunks;
  int64_t chunk = ceil_div(s.n, cs);
  chunk = ceil_div(chunk, 256 * VEC) * (256 * VEC);
  cs = ceil_div(s.n, chunk);
  s.fwd_chunk = chunk;
  s.fwd_chunks = (int)cs;
  fwd = BGrid{0, (int)cs, (int)rb, 1};
}

}  // namespace

bool b_aligned16(const void* p, int64_t ld, int dtype) { return aligned16(p, ld, dtype_size(dtype)); }

void b_plan_gram_res(int dtype, BSys& s) {
  const int64_t es = dtype_size(dtype);
  const int64_t cpt = 32 / es > 0 ? 32 / es : 1;
  s.res_nstrips = ceil_div(s.n, 8 * cpt);
  s.res_spw = ceil_div(s.res_nstrips, (int64_t)s.gram_G);
}

int b_plan_gram(int bulk_dtype, BSys& s, BGrid& gram, BGrid& red) {
  switch (bulk_dtype) {
    case 0: return plan_gram_t<cd>(s, gram, red);
    case 1: return plan_gram_t<cf>(s, gram, red);
    case 2: return plan_gram_t<double>(s, gram, red);
    default: return plan_gram_t<float>(s, gram, red);
  }
}

void b_plan_wide(int dtype, bool aligned, BSys& s, BGrid& adj, BGrid& sum, BGrid& fwd) {
  switch (dtype) {
    case 0: plan_wide_t<cd>(aligned, s, adj, sum, fwd); break;
    case 1: plan_wide_t<cf>(aligned, s, adj, sum, fwd); break;
    case 2: plan_wide_t<double>(aligned, s, adj, sum, fwd); break;
    default: plan_wide_t<float>(aligned, s, adj, sum, fwd); break;
  }
}

template <typename V, typename C, typename U, int RPT>
static void b_gram_one(const BLaunch& L, int mode, hipStream_t st) {
  constexpr int CPT = 32 / (int)sizeof(V) > 0 ? 32 / (int)sizeof(V) : 1;
  constexpr int CPTC = RPT == 1 ? 8 : 16 / RPT;
  if (L.total <= 0) return;
  if (mode == 1)
    hipLaunchKernelGGL((kb_gram_wt<V, C, U, CPT, RPT, Vec16<V>::n>), dim3((unsigned)L.total), dim3(512), 0, st, L.sys,
                       L.grid, L.nsys);
  else if (mode == 2)
    hipLaunchKernelGGL((kb_gram_cm<V, C, U, CPTC, RPT>), dim3((unsigned)L.total), dim3(512), 0, st, L.sys, L.grid,
                       L.nsys);
  else
    hipLaunchKernelGGL((kb_gram<V, C, U, CPT, RPT, Vec16<V>::n>), dim3((unsigned)L.total), dim3(512), 0, st, L.sys,
                       L.grid, L.nsys);
}

// Streams of the four rows-per-lane classes: with a fork, classes 1 .. 3
// that have work run on its side streams, which wait for an event recorded
// on st and are joined back into st by events of their own (under graph
// capture this records parallel branches); without, all run on st.
static hipError_t fork_out(const StreamFork* fk, const BLaunch* L, hipStream_t st, hipStream_t* s) {
  for (int k = 0; k < 4; ++k) s[k] = st;
  if (!fk) return hipSuccess;
  hipError_t e = hipEventRecord(fk->ev[0], st);
  for (int k = 1; k < 4 && e == hipSuccess; ++k)
    if (L[k].total > 0) {
      e = hipStreamWaitEvent(fk->side[k - 1], fk->ev[0], 0);
      s[k] = fk->side[k - 1];
    }
  return e;
}
static hipError_t fork_in(const StreamFork* fk, hipStream_t st, const hipStream_t* s) {
  hipError_t e = hipSuccess;
  for (int k = 1; k < 4 && e == hipSuccess; ++k)
    if (s[k] != st) {
      e = hipEventRecord(fk->ev[k], s[k]);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, fk->ev[k], 0);
    }
  return e;
}

template <typename V, typename C, typename U>
static hipError_t b_gram_go(const BLaunch* L, const BLaunch& red, int mode, hipStream_t st, const StreamFork* fk) {
  hipStream_t s[4];
  hipError_t e = fork_out(fk, L, st, s);
  if (e != hipSuccess) return e;
  b_gram_one<V, C, U, 1>(L[0], mode, s[0]);
  b_gram_one<V, C, U, 2>(L[1], mode, s[1]);
  b_gram_one<V, C, U, 4>(L[2], mode, s[2]);
  b_gram_one<V, C, U, 8>(L[3], mode, s[3]);
  if ((e = hipGetLastError()) != hipSuccess || (e = fork_in(fk, st, s)) != hipSuccess) return e;
  if (red.total > 0)
    hipLaunchKernelGGL((kb_gram_reduce<U>), dim3((unsigned)red.total), dim3(256), 0, st, red.sys, red.grid,
                       red.nsys, 1);
  return hipGetLastError();
}

template <typename V, typename U, int RPT>
static void b_res_one(const BLaunch& L, hipStream_t st) {
  constexpr int CPT = 32 / (int)sizeof(V) > 0 ? 32 / (int)sizeof(V) : 1;
  if (L.total > 0)
    hipLaunchKernelGGL((kb_gram_res<V, U, CPT, RPT>), dim3((unsigned)L.total), dim3(512), 0, st, L.sys, L.grid,
                       L.nsys);
}

template <typename V, typename U>
static hipError_t b_res_go(const BLaunch* L, const BLaunch& red, hipStream_t st, const StreamFork* fk) {
  hipStream_t s[4];
  hipError_t e = fork_out(fk, L, st, s);
  if (e != hipSuccess) return e;
  b_res_one<V, U, 1>(L[0], s[0]);
  b_res_one<V, U, 2>(L[1], s[1]);
  b_res_one<V, U, 4>(L[2], s[2]);
  b_res_one<V, U, 8>(L[3], s[3]);
  if ((e = hipGetLastError()) != hipSuccess || (e = fork_in(fk, st, s)) != hipSuccess) return e;
  if (red.total > 0)
    hipLaunchKernelGGL((kb_gram_reduce<U>), dim3((unsigned)red.total), dim3(256), 0, st, red.sys, red.grid,
                       red.nsys, 0);
  return hipGetLastError();
}

hipError_t launch_b_gram_res(int dtype, const BLaunch* L, const BLaunch& red, hipStream_t st, const StreamFork* fk) {
  switch (dtype) {
    case 0: return b_res_go<cd, cd>(L, red, st, fk);
    case 1: return b_res_go<cf, cd>(L, red, st, fk);
    case 2: return b_res_go<double, double>(L, red, st, fk);
    case 3: return b_res_go<float, double>(L, red, st, fk);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_b_gram(int dtype, const BLaunch* L, const BLaunch& red, int mode, hipStream_t st,
                         const StreamFork* fk) {
  switch (dtype) {
    case 0: return b_gram_go<cd, cd, cd>(L, red, mode, st, fk);
    case 1: return b_gram_go<cf, cf, cd>(L, red, mode, st, fk);
    case 2: return b_gram_go<double, double, double>(L, red, mode, st, fk);
    case 3: return b_gram_go<float, float, double>(L, red, mode, st, fk);
  }
  return hipErrorInvalidValue;
}

template <typename V, typename W>
static hipError_t b_adj_go(bool aligned, const BLaunch& L, const BLaunch& sum, int use_y, int to_x, hipStream_t st) {
  if (L.total > 0) {
    if (aligned)
      hipLaunchKernelGGL((kb_adj<V, W, Vec16<V>::n>), dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid,
                         L.nsys, use_y);
    else
      hipLaunchKernelGGL((kb_adj<V, W, 1>), dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys, use_y);
  }
  if (sum.total > 0)
    hipLaunchKernelGGL((kb_sum_slabs<W>), dim3((unsigned)sum.total), dim3(256), 0, st, sum.sys, sum.grid, sum.nsys,
                       to_x);
  return hipGetLastError();
}

hipError_t launch_b_adj_wide(int dtype, bool aligned, const BLaunch& L, const BLaunch& sum, int use_y, int to_x,
                             hipStream_t st) {
  switch (dtype) {
    case 0: return b_adj_go<cd, cd>(aligned, L, sum, use_y, to_x, st);
    case 1: return b_adj_go<cf, cd>(aligned, L, sum, use_y, to_x, st);
    case 2: return b_adj_go<double, double>(aligned, L, sum, use_y, to_x, st);
    case 3: return b_adj_go<float, double>(aligned, L, sum, use_y, to_x, st);
  }
  return hipErrorInvalidValue;
}

template <typename V, typename W>
static hipError_t b_fwd_go(bool aligned, const BLaunch& L, hipStream_t st) {
  if (L.total > 0) {
    if (aligned)
      hipLaunchKernelGGL((kb_fwd<V, W, Vec16<V>::n>), dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid,
                         L.nsys);
    else
      hipLaunchKernelGGL((kb_fwd<V, W, 1>), dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys);
  }
  return hipGetLastError();
}

hipError_t launch_b_fwd_wide(int dtype, bool aligned, const BLaunch& L, hipStream_t st) {
  switch (dtype) {
    case 0: return b_fwd_go<cd, cd>(aligned, L, st);
    case 1: return b_fwd_go<cf, cd>(aligned, L, st);
    case 2: return b_fwd_go<double, double>(aligned, L, st);
    case 3: return b_fwd_go<float, double>(aligned, L, st);
  }
  return hipErrorInvalidValue;
}

// ------------------------- compensated FP64 passes ----------------------------
// For the refinement residual b - A (A* y) and x = A* y when cond(A) u64
// approaches eps (cancellation in the sums is then of order cond(A)): every
// dot product is accumulated in double-double (Ogita, Rump and Oishi 2005:
// TwoProd by FMA, TwoSum by Knuth's six additions), partial sums are kept as
// (hi, lo) pairs and folded with TwoSum, and each result is rounded once.
// Floating-point contraction is off inside these helpers: the error-free
// transformations need the products and sums exactly as written.
namespace {

struct ddv {
  double hi, lo;
};

__device__ inline void dd_add(ddv& a, double x) {
#pragma clang fp contract(off)
  const double s = a.hi + x;
  const double z = s - a.hi;
  const double e = (a.hi - (s - z)) + (x - z);
  a.hi = s;
  a.lo += e;
}
__device__ inline void dd_fma(ddv& a, double x, double y) {
#pragma clang fp contract(off)
  const double p = x * y;
  const double ep = fma(x, y, -p);
  dd_add(a, p);
  a.lo += ep;
}
__device__ inline void dd_merge(ddv& a, const ddv& b) {
#pragma clang fp contract(off)
  dd_add(a, b.hi);
  a.lo += b.lo;
}
__device__ inline double dd_round(const ddv& a) {
#pragma clang fp contract(off)
  return a.hi + a.lo;
}
__device__ inline ddv dd_shfl_xor(const ddv& a, int off) {
  return ddv{__shfl_xor(a.hi, off, 64), __shfl_xor(a.lo, off, 64)};
}

// complex or real accumulator: 2 (re, im) or 1 double-double
template <bool CPLX> struct Acc2 {
  ddv c[CPLX ? 2 : 1];
};

// acc += conj(a) u (adjoint) or a w (forward), a promoted to FP64
template <bool CONJ, typename V, typename W>
__device__ inline void acc_mac(Acc2<VT<W>::cplx>& acc, const V& a, const W& u) {
  if constexpr (VT<W>::cplx) {
    const double ar = (double)vre(a), ai = (double)vim(a), ur = vre(u), ui = vim(u);
    dd_fma(acc.c[0], ar, ur);
    dd_fma(acc.c[0], CONJ ? ai : -ai, ui);
    dd_fma(acc.c[1], ar, ui);
    dd_fma(acc.c[1], CONJ ? -ai : ai, ur);
  } else {
    dd_fma(acc.c[0], (double)vre(a), (double)vre(u));
  }
}

// w (hi/lo slab partials) = A* u.  grid (ceil(n / 256), RS), 256 threads.
template <typename V, typename W>
__global__ void __launch_bounds__(256) k_adj_dd(const V* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                const W* __restrict__ u, int64_t rows_per_slab, W* __restrict__ ph,
                                                W* __restrict__ pl) {
  constexpr bool C = VT<W>::cplx;
  __shared__ W su[1024];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_slab;
  const int64_t r1 = (r0 + rows_per_slab) < m ? (r0 + rows_per_slab) : m;
  Acc2<C> acc{};
  for (int64_t rb = r0; rb < r1; rb += 1024) {
    const int64_t rn = (r1 - rb) < 1024 ? (r1 - rb) : 1024;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < rn; t += 256) su[t] = u[rb + t];
    __syncthreads();
    if (j < n) {
      const V* a = A + rb * lda + j;
      int64_t i = 0;
      for (; i + 4 <= rn; i += 4) {
        V x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = ld_once(a + (i + k) * lda);
#pragma unroll
        for (int k = 0; k < 4; ++k) acc_mac<true>(acc, x[k], su[i + k]);
      }
      for (; i < rn; ++i) acc_mac<true>(acc, ld_once(a + i * lda), su[i]);
    }
  }
  if (j >= n) return;
  const int64_t o = (int64_t)blockIdx.y * n + j;
  if constexpr (C) {
    ph[o] = W{acc.c[0].hi, acc.c[1].hi};
    pl[o] = W{acc.c[0].lo, acc.c[1].lo};
  } else {
    ph[o] = acc.c[0].hi;
    pl[o] = acc.c[0].lo;
  }
}

// w[j] = sum over slabs of (hi + lo), compensated, rounded once.
template <typename W>
__global__ void __launch_bounds__(256) k_sum_dd(const W* __restrict__ ph, const W* __restrict__ pl, int rs, int64_t n,
                                                W* __restrict__ w) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  ddv re{0.0, 0.0}, im{0.0, 0.0};
  for (int k = 0; k < rs; ++k) {
    const W h = ph[(int64_t)k * n + j], l = pl[(int64_t)k * n + j];
    dd_merge(re, ddv{vre(h), vre(l)});
    if constexpr (VT<W>::cplx) dd_merge(im, ddv{vim(h), vim(l)});
  }
  w[j] = vmake<W>(dd_round(re), dd_round(im));
}

// (hi, lo) chunk partials of q = A w.  grid (CS, ceil(m / RB)), 256 threads.
template <typename V, typename W, int RB>
__global__ void __launch_bounds__(256) k_fwd_dd(const V* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                const W* __restrict__ w, int64_t chunk, W* __restrict__ qh,
                                                W* __restrict__ ql) {
  constexpr bool C = VT<W>::cplx;
  constexpr int NC = C ? 2 : 1;
  __shared__ ddv red[RB][NC][4];
  const int64_t i0 = (int64_t)blockIdx.y * RB;
  const int64_t c0 = (int64_t)blockIdx.x * chunk;
  const int64_t c1 = (c0 + chunk) < n ? (c0 + chunk) : n;
  int64_t rows = m - i0;
  if (rows > RB) rows = RB;
  Acc2<C> acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = Acc2<C>{};
  for (int64_t j = c0 + threadIdx.x; j < c1; j += 256) {
    const W wj = w[j];
#pragma unroll
    for (int r = 0; r < RB; ++r)
      if (r < rows) acc_mac<false>(acc[r], ld_once(A + (i0 + r) * lda + j), wj);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      ddv v = acc[r].c[c];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) dd_merge(v, dd_shfl_xor(v, off));
      if (lane == 0) red[r][c][wv] = v;
    }
  __syncthreads();
  if (threadIdx.x < RB && threadIdx.x < rows) {
    const int r = threadIdx.x;
    ddv v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      v[c] = red[r][c][0];
      for (int k = 1; k < 4; ++k) dd_merge(v[c], red[r][c][k]);
    }
    const int64_t o = (int64_t)blockIdx.x * m + i0 + r;
    if constexpr (C) {
      qh[o] = W{v[0].hi, v[1].hi};
      ql[o] = W{v[0].lo, v[1].lo};
    } else {
      qh[o] = v[0].hi;
      ql[o] = v[0].lo;
    }
  }
}

template <typename W>
__global__ void __launch_bounds__(256) k_fold_dd(const W* __restrict__ qh, const W* __restrict__ ql, int cs, int64_t m,
                                                 W* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  ddv re{0.0, 0.0}, im{0.0, 0.0};
  for (int k = 0; k < cs; ++k) {
    const W h = qh[(int64_t)k * m + i], l = ql[(int64_t)k * m + i];
    dd_merge(re, ddv{vre(h), vre(l)});
    if constexpr (VT<W>::cplx) dd_merge(im, ddv{vim(h), vim(l)});
  }
  q[i] = vmake<W>(dd_round(re), dd_round(im));
}

template <typename V, typename W>
hipError_t adj_dd_impl(const AdjArgs& a, hipStream_t st) {
  const int64_t nb = ceil_div(a.n, (int64_t)256);
  const int64_t rs = slabs_for(a.m, a.n, 1);
  const int64_t rps = ceil_div(a.m, rs);
  W* ph = reinterpret_cast<W*>(a.part);
  W* pl = ph + rs * a.n;
  hipLaunchKernelGGL((k_adj_dd<V, W>), dim3((unsigned)nb, (unsigned)rs), dim3(256), 0, st,
                     reinterpret_cast<const V*>(a.A), a.lda, a.m, a.n, reinterpret_cast<const W*>(a.u), rps, ph, pl);
  hipLaunchKernelGGL((k_sum_dd<W>), dim3((unsigned)ceil_div(a.n, 256)), dim3(256), 0, st, ph, pl, (int)rs, a.n,
                     reinterpret_cast<W*>(a.w));
  return hipGetLastError();
}

template <typename V, typename W>
hipError_t fwd_dd_impl(const FwdArgs& a, void* q, hipStream_t st) {
  constexpr int RB = 8;
  const int64_t rb = ceil_div(a.m, RB);
  int64_t cs = ceil_div(2048, rb);
  if (cs > ceil_div(a.n, 512)) cs = ceil_div(a.n, 512);
  if (cs < 1) cs = 1;
  if (cs > kMaxChunks / 2) cs = kMaxChunks / 2;
  int64_t chunk = ceil_div(a.n, cs);
  chunk = ceil_div(chunk, 256) * 256;
  cs = ceil_div(a.n, chunk);
  W* qh = reinterpret_cast<W*>(a.qpart);
  W* ql = qh + cs * a.m;
  hipLaunchKernelGGL((k_fwd_dd<V, W, RB>), dim3((unsigned)cs, (unsigned)rb), dim3(256), 0, st,
                     reinterpret_cast<const V*>(a.A), a.lda, a.m, a.n, reinterpret_cast<const W*>(a.w), chunk, qh,
                     ql);
  hipLaunchKernelGGL((k_fold_dd<W>), dim3((unsigned)ceil_div(a.m, 256)), dim3(256), 0, st, qh, ql, (int)cs, a.m,
                     reinterpret_cast<W*>(q));
  if (a.chunks_out) *a.chunks_out = 1;
  return hipGetLastError();
}

}  // namespace

int64_t adj_dd_part_elems(int64_t m, int64_t n) { return 2 * slabs_for(m, n, 1) * n; }

hipError_t launch_gemv_adj_dd(int dtype, const AdjArgs& a, hipStream_t st) {
  switch (dtype) {
    case 0: return adj_dd_impl<cd, cd>(a, st);
    case 1: return adj_dd_impl<cf, cd>(a, st);
    case 2: return adj_dd_impl<double, double>(a, st);
    case 3: return adj_dd_impl<float, double>(a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemv_fwd_dd(int dtype, const FwdArgs& a, void* q, hipStream_t st) {
  switch (dtype) {
    case 0: return fwd_dd_impl<cd, cd>(a, q, st);
    case 1: return fwd_dd_impl<cf, cd>(a, q, st);
    case 2: return fwd_dd_impl<double, double>(a, q, st);
    case 3: return fwd_dd_impl<float, double>(a, q, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace mn
