// Step 1 of the method (eq. randmat): S = T A*, T = S F D, applied to every
// row of A with a radix-staged FFT in LDS.
//
//   row i:  v = d o conj(a_i) zero-padded to N;  V = F v;  S(k, i) = V[idx[k]]
//
// F is the unitary DFT of eq. (DFT), entries N^{-1/2} exp(-2 pi i j k / N).
// For real data F is replaced by the orthonormal Hartley transform (the
// paper's "real-valued version"): the row is transformed as a complex
// sequence with zero imaginary part and Re(V) - Im(V) is kept.
//
// Two launch shapes:
//   * N <= LDS limit: one workgroup transforms B whole rows in LDS.
//   * larger N = N1 * N2 ("four-step"): pass 1 does the N2-point FFTs down
//     the columns of the N2 x N1 view of each row and multiplies by the
//     twiddles W_N^{n1 k2}; pass 2 does the N1-point FFTs along the rows of
//     the intermediate and scatters the kept outputs into S through the
//     inverse subsample map.
// The twiddle table holds W_N^k (k < N) followed by compact tables W_{N1}^k
// (k < N1) for the splits N1 = N1_0, 2 N1_0, 4 N1_0 (N1_0 = N / 2^floor(log2(N)/2)):
// the four-step stages and the W_N^{n1 k2} = W_N^{rem} W_{N2}^{q} factors
// (n1 k2 = q N1 + rem) read only the first N1 entries and one compact
// table, small enough to stay in cache.  A split with a shorter N2 gives
// pass 1 longer contiguous row segments (4096 / N2 elements).
// Both use the same batched Stockham FFT: 256 threads, 16 elements per
// thread, radix-16/8/4/2 butterflies in registers, LDS between stages.
#include "common.hpp"
#include "kernels.hpp"
#include "batch_dev.hpp"

namespace mn {

// ---------------------------------------------------------------------------
// in-register DFTs, forward sign:  X[k] = sum_r v[r] exp(-2 pi i r k / R)
// ---------------------------------------------------------------------------
template <typename C> __device__ inline void dft2(C& a, C& b) {
  C t = a;
  a = vadd(t, b);
  b = vsub(t, b);
}

template <typename C> __device__ inline void dft4(C& v0, C& v1, C& v2, C& v3) {
  C t0 = vadd(v0, v2), t1 = vsub(v0, v2);
  C t2 = vadd(v1, v3), t3 = vmul_negi(vsub(v1, v3));
  v0 = vadd(t0, t2);
  v2 = vsub(t0, t2);
  v1 = vadd(t1, t3);
  v3 = vsub(t1, t3);
}

// multiply by W_16^e = exp(-2 pi i e / 16); e is a compile-time constant
template <int E, typename C> __device__ inline C w16(C a) {
  constexpr int e = E & 15;
  if constexpr (e == 0) return a;
  else if constexpr (e == 4) return vmul_negi(a);
  else if constexpr (e == 8) return vscale(a, (typename VT<C>::real)(-1));
  else if constexpr (e == 12) return C{-a.im, a.re};
  else {
    using R = typename VT<C>::real;
    // cos(2 pi e/16) and sin(2 pi e/16) via quarter-wave symmetry
    constexpr int q = e & 3;      // offset within the quadrant
    constexpr int quad = e >> 2;  // quadrant
    const R c0 = (R)(q == 1 ? 0.92387953251128675613 : q == 2 ? 0.70710678118654752440 : 0.38268343236508977173);
    const R s0 = (R)(q == 1 ? 0.38268343236508977173 : q == 2 ? 0.70710678118654752440 : 0.92387953251128675613);
    R c, s;
    if constexpr (quad == 0) { c = c0; s = s0; }
    else if constexpr (quad == 1) { c = -s0; s = c0; }
    else if constexpr (quad == 2) { c = -c0; s = -s0; }
    else { c = s0; s = -c0; }
    // (a.re + i a.im) * (c - i s)
    return C{a.re * c + a.im * s, a.im * c - a.re * s};
  }
}

// 8 = 2 x 4: r = r2 + 4 r1, k = k1 + 2 k2.  Output X[k] is left in
// v[perm8(k)] = v[4 (k % 2) + k / 2].
template <typename C> __device__ inline void dft8(C* v) {
#pragma unroll
  for (int r2 = 0; r2 < 4; ++r2) dft2(v[r2], v[r2 + 4]);
  v[5] = w16<2>(v[5]);
  v[6] = w16<4>(v[6]);
  v[7] = w16<6>(v[7]);
  dft4(v[0], v[1], v[2], v[3]);
  dft4(v[4], v[5], v[6], v[7]);
}

// 16 = 4 x 4: r = r2 + 4 r1, k = k1 + 4 k2.  Output X[k] is left in
// v[perm16(k)] = v[4 (k % 4) + k / 4].
template <typename C> __device__ inline void dft16(C* v) {
#pragma unroll
  for (int r2 = 0; r2 < 4; ++r2) dft4(v[r2], v[r2 + 4], v[r2 + 8], v[r2 + 12]);
  // now v[r2 + 4 k1] holds u[r2][k1]; twiddle W16^{r2 k1}
  v[5] = w16<1>(v[5]);
  v[6] = w16<2>(v[6]);
  v[7] = w16<3>(v[7]);
  v[9] = w16<2>(v[9]);
  v[10] = w16<4>(v[10]);
  v[11] = w16<6>(v[11]);
  v[13] = w16<3>(v[13]);
  v[14] = w16<6>(v[14]);
  v[15] = w16<9>(v[15]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
}

// register slot holding output k of a radix-R butterfly
template <int R> __host__ __device__ constexpr int out_slot(int k) {
  return R == 16 ? 4 * (k % 4) + k / 4 : (R == 8 ? 4 * (k % 2) + k / 2 : k);
}

template <int R, typename C> __device__ inline void dftR(C* v) {
  if constexpr (R == 2) dft2(v[0], v[1]);
  else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8(v);
  else if constexpr (R == 16) dft16(v);
}

// LDS index with one padding element every 16 (breaks power-of-two strides)
__device__ inline int lpad(int i) { return i + (i >> 4); }
__host__ __device__ inline int lds_stride(int L) { return L + (L >> 4) + 1; }

// One Stockham stage of radix R for the FFT owned by this thread.
//   L   transform length, Ns product of the radices already applied,
//   tpf threads per FFT, tl this thread's index within its FFT,
//   tw  table of W_Nt^k, k < Nt, twm = Nt / L.
// All sizes are powers of two: index arithmetic uses shifts and masks of the
// (wave-uniform) base-2 logarithms rather than integer division.
template <int R, typename C>
__device__ inline void fft_stage(C* buf, int L, int Ns, int tpf, int tl, const C* __restrict__ tw, int twm) {
  constexpr int SMAX = 16 / R;
  constexpr int LGR = R == 16 ? 4 : (R == 8 ? 3 : (R == 4 ? 2 : 1));
  const int lgL = __builtin_ctz((unsigned)L), lgNs = __builtin_ctz((unsigned)Ns);
  const int lgtpf = __builtin_ctz((unsigned)tpf), lgtwm = __builtin_ctz((unsigned)twm);
  const int slots = L >> (LGR + lgtpf);  // 16 / R when E = 16
  const int LR = L >> LGR;
  // W_{Ns R}^{r jm} = W_Nt^{r jm Nt/(Ns R)}, Nt / (Ns R) = (L / (Ns R)) twm
  const int lge = lgL - lgNs - LGR + lgtwm;
  C v[16];
#pragma unroll
  for (int s = 0; s < SMAX; ++s) {
    if (s < slots && tl < tpf) {
      const int j = tl + (s << lgtpf);
      const int jm = j & (Ns - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C x = buf[lpad(j + r * LR)];
        if (r > 0 && jm > 0) x = vmul(x, tw[(r * jm) << lge]);
        v[s * R + r] = x;
      }
      dftR<R>(v + s * R);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SMAX; ++s) {
    if (s < slots && tl < tpf) {
      const int j = tl + (s << lgtpf);
      const int jm = j & (Ns - 1);
      const int d0 = ((j >> lgNs) << (lgNs + LGR)) + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lpad(d0 + (r << lgNs))] = v[s * R + out_slot<R>(r)];
    }
  }
  __syncthreads();
}

// Full FFT of length L (power of two) on buf[lpad(0..L)), done by tpf threads.
// Requires a __syncthreads() before the call (data in place).
template <typename C>
__device__ inline void fft_lds(C* buf, const FftPlan& pl, int tpf, int tl, const C* __restrict__ tw, int twm) {
  int Ns = 1;
  for (int s = 0; s < pl.nst; ++s) {
    const int R = pl.radix[s];
    if (R == 16) fft_stage<16>(buf, pl.L, Ns, tpf, tl, tw, twm);
    else if (R == 8) fft_stage<8>(buf, pl.L, Ns, tpf, tl, tw, twm);
    else if (R == 4) fft_stage<4>(buf, pl.L, Ns, tpf, tl, tw, twm);
    else fft_stage<2>(buf, pl.L, Ns, tpf, tl, tw, twm);
    Ns *= R;
  }
}

// value of the padded, phase-multiplied row entry: d_j conj(a_j) (complex)
// or d_j a_j + 0i (real)
template <typename V, typename C>
__device__ inline C load_row_entry(const V* __restrict__ row, int64_t j, int64_t n, const void* __restrict__ dv) {
  if (j >= n) return vzero<C>();
  if constexpr (VT<V>::cplx) {
    const cd dd = reinterpret_cast<const cd*>(dv)[j];
    const C d = vmake<C>(dd.re, dd.im);
    return vcmul(vconv<C>(row[j]), d);  // conj(a) * d
  } else {
    const double dd = reinterpret_cast<const double*>(dv)[j];
    using R = typename VT<C>::real;
    return C{(R)row[j] * (R)dd, (R)0};
  }
}

template <typename V, typename C>
__device__ inline V out_value(C x, typename VT<C>::real scale) {
  if constexpr (VT<V>::cplx) return vconv<V>(vscale(x, scale));
  else return (V)((x.re - x.im) * scale);
}

// --------------------------- whole rows in LDS ------------------------------
// grid.x = ceil(m / B); B rows per workgroup, 256 threads.
template <typename V, typename C>
__device__ __forceinline__ void k_sketch_small_body(const Bk bk, const V* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                      FftPlan pl, int B, const void* __restrict__ d,
                                                      const int32_t* __restrict__ idx, int64_t l,
                                                      V* __restrict__ S, int64_t lds, const C* __restrict__ tw,
                                                      typename VT<C>::real scale) {
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const int L = pl.L;
  const int lgL = __builtin_ctz((unsigned)L);
  const int Lp = lds_stride(L);
  const int E = L < 16 ? L : 16;
  const int tpf = L / E;
  const int lgtpf = __builtin_ctz((unsigned)tpf);
  const int64_t row0 = (int64_t)bk.x * B;
  // load: consecutive threads read consecutive entries of one row; all of a
  // thread's loads are issued before any is used
  {
    C v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = threadIdx.x + u * 256;
      const int b = t >> lgL, pos = t & (L - 1);
      const int64_t i = row0 + b;
      v[u] = (t < B * L && i < m) ? load_row_entry<V, C>(A + i * lda, pos, n, d) : vzero<C>();
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = threadIdx.x + u * 256;
      if (t < B * L) sm[(t >> lgL) * Lp + lpad(t & (L - 1))] = v[u];
    }
  }
  __syncthreads();
  const int b = threadIdx.x >> lgtpf, tl = threadIdx.x & (tpf - 1);
  const bool active = b < B;
  {
    // every thread must reach the stage barriers: inactive threads work on a
    // harmless private copy of FFT 0's index range but write nothing back
    C* buf = sm + (active ? b : 0) * Lp;
    int Ns = 1;
    for (int s = 0; s < pl.nst; ++s) {
      const int R = pl.radix[s];
      const int tl_eff = active ? tl : tpf;  // tl = tpf -> no slots executed
      if (R == 16) fft_stage<16>(buf, L, Ns, tpf, tl_eff, tw, 1);
      else if (R == 8) fft_stage<8>(buf, L, Ns, tpf, tl_eff, tw, 1);
      else if (R == 4) fft_stage<4>(buf, L, Ns, tpf, tl_eff, tw, 1);
      else fft_stage<2>(buf, L, Ns, tpf, tl_eff, tw, 1);
      Ns *= R;
    }
  }
  // gather the kept outputs: column i of S
  for (int bb = 0; bb < B; ++bb) {
    const int64_t i = row0 + bb;
    if (i >= m) break;
    for (int64_t k = threadIdx.x; k < l; k += blockDim.x) {
      const int pos = idx[k];
      S[k + i * lds] = out_value<V, C>(sm[bb * Lp + lpad(pos)], scale);
    }
  }
}
template <typename V, typename C>
__global__ void __launch_bounds__(256) k_sketch_small(const V* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                      FftPlan pl, int B, const void* __restrict__ d,
                                                      const int32_t* __restrict__ idx, int64_t l,
                                                      V* __restrict__ S, int64_t lds, const C* __restrict__ tw,
                                                      typename VT<C>::real scale) {
  k_sketch_small_body<V, C>(bk_hw(), A, lda, m, n, pl, B, d, idx, l, S, lds, tw, scale);
}

// ----------------------- four-step, pass 1: columns -------------------------
// Row i viewed as N2 x N1 (x[n1 + N1 n2]); FFT over n2 for B consecutive n1,
// times W_N^{n1 k2}; writes Y[i][k2][n1].  grid = (N1 / B, rows in chunk).
template <typename V, typename C>
__device__ __forceinline__ void k_sketch_cols_body(const Bk bk, const V* __restrict__ A, int64_t lda, int64_t row0, int64_t m,
                                                     int64_t n, int N1, FftPlan pl2, int B,
                                                     const void* __restrict__ d, C* __restrict__ Y,
                                                     const C* __restrict__ tw, const C* __restrict__ twc) {
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const int N2 = pl2.L;
  const int Lp = lds_stride(N2);
  const int64_t i = row0 + bk.y;
  const int c0 = bk.x * B;
  const int64_t N = (int64_t)N1 * N2;
  const int lgB = __builtin_ctz((unsigned)B);
  const V* row = A + i * lda;
  // load: consecutive threads take consecutive n1 (contiguous in memory);
  // B * N2 <= 4096 = 16 per thread, all issued before use
  {
    C v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = threadIdx.x + u * 256;
      const int bb = t & (B - 1), n2 = t >> lgB;
      const int64_t j = (int64_t)(c0 + bb) + (int64_t)N1 * n2;
      v[u] = (t < B * N2 && i < m) ? load_row_entry<V, C>(row, j, n, d) : vzero<C>();
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = threadIdx.x + u * 256;
      if (t < B * N2) sm[(t & (B - 1)) * Lp + lpad(t >> lgB)] = v[u];
    }
  }
  __syncthreads();
  const int E = N2 < 16 ? N2 : 16;
  const int tpf = N2 / E;
  const int lgtpf = __builtin_ctz((unsigned)tpf);
  const int b = threadIdx.x >> lgtpf, tl = threadIdx.x & (tpf - 1);
  const bool active = b < B;
  C* buf = sm + (active ? b : 0) * Lp;
  {
    int Ns = 1;
    const int twm = N1 / N2;  // W_N2^k = W_N1^{k N1 / N2}
    for (int s = 0; s < pl2.nst; ++s) {
      const int R = pl2.radix[s];
      const int tl_eff = active ? tl : tpf;
      if (R == 16) fft_stage<16>(buf, N2, Ns, tpf, tl_eff, twc, twm);
      else if (R == 8) fft_stage<8>(buf, N2, Ns, tpf, tl_eff, twc, twm);
      else if (R == 4) fft_stage<4>(buf, N2, Ns, tpf, tl_eff, twc, twm);
      else fft_stage<2>(buf, N2, Ns, tpf, tl_eff, twc, twm);
      Ns *= R;
    }
  }
  if (i >= m) return;
  // twiddle W_N^{n1 k2} and store Y[i][k2][n1]: consecutive threads, consecutive n1
  C* Yi = Y + (int64_t)bk.y * N;
  const int lg1 = __builtin_ctz((unsigned)N1);
  const unsigned r12 = (unsigned)(N1 / N2);
  C wv[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int t = threadIdx.x + u * 256;
    const unsigned e = (unsigned)(c0 + (t & (B - 1))) * (unsigned)(t >> lgB);  // n1 k2 < N
    // W_N^e = W_N^{e mod N1} W_N2^{floor(e / N1)}
    wv[u] = (t < B * N2) ? vmul(tw[e & (unsigned)(N1 - 1)], twc[(e >> lg1) * r12]) : vzero<C>();
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int t = threadIdx.x + u * 256;
    if (t < B * N2) {
      const int bb = t & (B - 1), k2 = t >> lgB;
      Yi[(int64_t)k2 * N1 + c0 + bb] = vmul(sm[bb * Lp + lpad(k2)], wv[u]);
    }
  }
}
template <typename V, typename C>
__global__ void __launch_bounds__(256) k_sketch_cols(const V* __restrict__ A, int64_t lda, int64_t row0, int64_t m,
                                                     int64_t n, int N1, FftPlan pl2, int B,
                                                     const void* __restrict__ d, C* __restrict__ Y,
                                                     const C* __restrict__ tw, const C* __restrict__ twc) {
  k_sketch_cols_body<V, C>(bk_hw(), A, lda, row0, m, n, N1, pl2, B, d, Y, tw, twc);
}

// ---------------------- four-step, pass 2: rows + gather ---------------------
// FFT over n1 of Y[i][k2][:] for B consecutive k2; output index k = k2 + N2 k1
// is kept when inv[k] >= 0, written to S(inv[k], i).  grid = (N2 / B, rows).
template <typename V, typename C>
__device__ __forceinline__ void k_sketch_rows_body(const Bk bk, const C* __restrict__ Y, int64_t row0, int64_t m, int N2,
                                                     FftPlan pl1, int B, const int32_t* __restrict__ inv,
                                                     V* __restrict__ S, int64_t lds, const C* __restrict__ tw,
                                                     typename VT<C>::real scale) {
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const int N1 = pl1.L;
  const int Lp = lds_stride(N1);
  const int64_t N = (int64_t)N1 * N2;
  const int64_t i = row0 + bk.y;
  const int c0 = bk.x * B;
  const int lgN1 = __builtin_ctz((unsigned)N1);
  const C* Yi = Y + (int64_t)bk.y * N;
  {
    // rows c0 .. c0 + B - 1 of the N2 x N1 intermediate are contiguous
    const C* blk = Yi + (int64_t)c0 * N1;
    C v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = threadIdx.x + u * 256;
      v[u] = (t < B * N1 && i < m) ? blk[t] : vzero<C>();
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = threadIdx.x + u * 256;
      if (t < B * N1) sm[(t >> lgN1) * Lp + lpad(t & (N1 - 1))] = v[u];
    }
  }
  __syncthreads();
  const int E = N1 < 16 ? N1 : 16;
  const int tpf = N1 / E;
  const int lgtpf = __builtin_ctz((unsigned)tpf);
  const int b = threadIdx.x >> lgtpf, tl = threadIdx.x & (tpf - 1);
  const bool active = b < B;
  C* buf = sm + (active ? b : 0) * Lp;
  {
    int Ns = 1;
    const C* twc = tw;  // W_{N1}^k, k < N1
    for (int s = 0; s < pl1.nst; ++s) {
      const int R = pl1.radix[s];
      const int tl_eff = active ? tl : tpf;
      if (R == 16) fft_stage<16>(buf, N1, Ns, tpf, tl_eff, twc, 1);
      else if (R == 8) fft_stage<8>(buf, N1, Ns, tpf, tl_eff, twc, 1);
      else if (R == 4) fft_stage<4>(buf, N1, Ns, tpf, tl_eff, twc, 1);
      else fft_stage<2>(buf, N1, Ns, tpf, tl_eff, twc, 1);
      Ns *= R;
    }
  }
  if (i >= m) return;
  int32_t pos[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int t = threadIdx.x + u * 256;
    pos[u] = (t < B * N1) ? inv[(int64_t)(c0 + (t >> lgN1)) + (int64_t)N2 * (t & (N1 - 1))] : -1;
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int t = threadIdx.x + u * 256;
    if (pos[u] >= 0) S[pos[u] + i * lds] = out_value<V, C>(sm[(t >> lgN1) * Lp + lpad(t & (N1 - 1))], scale);
  }
}
template <typename V, typename C>
__global__ void __launch_bounds__(256) k_sketch_rows(const C* __restrict__ Y, int64_t row0, int64_t m, int N2,
                                                     FftPlan pl1, int B, const int32_t* __restrict__ inv,
                                                     V* __restrict__ S, int64_t lds, const C* __restrict__ tw,
                                                     typename VT<C>::real scale) {
  k_sketch_rows_body<V, C>(bk_hw(), Y, row0, m, N2, pl1, B, inv, S, lds, tw, scale);
}

// ------------------ four-step, kept outputs only (pruned) ---------------------
// Only l of the N outputs of each row's transform are kept.  With the input
// index n = n1 + N1 n2 (n1 < N1, n2 < N2) and an output k,
//   V[k] = sum_{n1} W_N^{n1 k} Z_{n1}[k mod N2],
//   Z_{n1}[k2] = sum_{n2} v[n1 + N1 n2] W_{N2}^{n2 k2}
// since W_N^{N1 n2 k} = W_{N2}^{n2 k}.  A workgroup takes one row and G
// blocks of B consecutive n1: it transforms the block's B columns in LDS
// (N2 = 16 TPB / B points each: 4096 / B with 256 threads, 8192 / B with
// the wide 512-thread form, 2048 at B = 4; the first radix-16 stage
// runs on the loaded registers) and adds the block's share of the outer sum
// to one register accumulator per kept output.  Neither the N2 x N1
// intermediate nor the discarded outputs reach memory; the outer sum costs
// l N1 = l N / N2 multiply-adds per row, so with N2 near l (the wide form)
// the row costs O(N log N2) for the column transforms plus about 8 N flops
// for the outer sum: O(N log l).  The outer sum is a polynomial in W_N^k
// with the values Z_{n1}[k mod N2] as coefficients, evaluated by Horner's
// rule on two levels: within a block (variable W_N^k, one complex
// multiply-add per column) and across the blocks, taken in decreasing order
// (variable W_N^{B k}, one more per block); a column group that starts at
// column cbeg multiplies its sum by W_N^{cbeg k} once at the end.  The two
// variables of every kept output come from a table laid out in slot order
// (k_sketch_steps), so each block reads them coalesced instead of gathering
// from the twiddle table.  Thread slot
// q = tid + TPB u takes kept output order[q]: the order groups outputs of
// equal k mod N2 (k_sketch_order), so the lanes of a wave read a few LDS
// addresses (broadcast) rather than 64 scattered ones.  With one column
// group per row (grid.x = 1) the workgroup writes S; otherwise the group's
// sums go to P[g][row][s] and k_sketch_fold adds them.  KPT = kept outputs
// per thread (2, 4, 8; with FP32 accumulators also 16 and 32).

// one-touch load of a streamed operand
template <typename V> __device__ __forceinline__ V ld_stream(const V* p) {
  if constexpr (VT<V>::cplx) {
    using Rl = typename VT<V>::real;
    const Rl* q = reinterpret_cast<const Rl*>(p);
    return V{__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1)};
  } else {
    return __builtin_nontemporal_load(p);
  }
}

// an LDS entry as one 8-byte (complex float) or 16-byte read: with the
// alignment stated, the constant column offsets fold into the instruction
template <typename C> __device__ __forceinline__ C lds_c(const C* p) {
  if constexpr (std::is_same<C, cf>::value) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    return cf{v.x, v.y};
  } else {
    return *p;
  }
}

// the kept-output table (2 l entries of the compute type) that follows the
// order's l indices in the same buffer (sketch_order_bytes)
template <typename C> __host__ __device__ inline const C* kept_steps(const int32_t* order, int64_t l) {
  return reinterpret_cast<const C*>(reinterpret_cast<const char*>(order) + ((4 * l + 255) & ~(int64_t)255));
}

template <typename V> struct PhaseOf { using type = typename std::conditional<VT<V>::cplx, cd, double>::type; };

template <int X> __host__ __device__ constexpr int ilog2c() { return X <= 1 ? 0 : 1 + ilog2c<X / 2>(); }

// Whether the kept-outputs-only form keeps its stage twiddles W_{N2}^k in LDS
// after the B columns: with 256 threads where two workgroups still fit a CU
// (B = 16, 8); with wider workgroups (one per CU) where the 160 KB hold both.
template <typename C, int B, int TPB> __host__ __device__ constexpr bool pruned_tw_lds() {
  constexpr int N2 = TPB * 16 / B;
  constexpr int64_t cols = (int64_t)B * (N2 + N2 / 16 + 1) * (int64_t)sizeof(C);
  constexpr int64_t with_tw = cols + (int64_t)N2 * (int64_t)sizeof(C);
  // wide form: where the table still leaves two workgroups to a CU, or where
  // the columns alone already take one CU
  return TPB == 256 ? B >= 8 : (with_tw <= 80 * 1024 || (cols > 80 * 1024 && with_tw <= 160 * 1024));
}

// bk.x = column group, bk.y = row within the launch, bk.gx = groups per row.
// TPB threads hold 16 elements each: N2 = 16 TPB / B points per column.
template <typename V, typename C, int B, int KPT, int TPB = 256>
__device__ __forceinline__ void k_sketch_pruned_body(const Bk bk, const V* __restrict__ A, int64_t lda, int64_t row0,
                                                       int64_t rows, int64_t n, int N1, int G, FftPlan pl2,
                                                       const void* __restrict__ dv, const int32_t* __restrict__ idx,
                                                       const int32_t* __restrict__ order, int64_t l,
                                                       const C* __restrict__ tw, V* __restrict__ S, int64_t lds,
                                                       C* __restrict__ P, typename VT<C>::real scale) {
  constexpr int N2 = TPB * 16 / B;
  constexpr int LR = N2 / 16;  // = TPB / B: butterflies per column in a radix-16 stage
  constexpr int lgB = ilog2c<B>(), lgLR = ilog2c<LR>();
  constexpr int Lp = N2 + N2 / 16 + 1;
  using D = typename PhaseOf<V>::type;
  using R = typename VT<C>::real;
  // the stage twiddles W_{N2}^k (k < N2) sit in LDS after the B columns
  // where they fit (pruned_tw_lds); otherwise the stages read W_N
  constexpr bool TW_LDS = pruned_tw_lds<C, B, TPB>();
  extern __shared__ unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  // N = N1 N2 with N2 a power of two and N1 any positive integer
  const uint64_t Ntot = (uint64_t)N1 * (uint64_t)N2;
  const int64_t i = row0 + bk.y;
  const V* row = A + i * lda;
  C* tws = sm + B * Lp;
  if constexpr (TW_LDS) {
    for (int k = threadIdx.x; k < N2; k += TPB) tws[k] = tw[(unsigned)k * (unsigned)N1];
  }
  const C* twst = TW_LDS ? tws : tw;
  const int twm = TW_LDS ? 1 : N1;
  const D* dp = reinterpret_cast<const D*>(dv);
  const int tid = threadIdx.x;
  // first stage and loads: column bb of the block, butterfly jj (inputs jj + r LR)
  const int bb = tid & (B - 1), jj = tid >> lgB;
  // later stages: column fb, thread tl of its LR
  const int fb = tid >> lgLR, tl = tid & (LR - 1);

  // kept output of slot u (slots past l compute on k = 0 and store nothing:
  // no branch in the sum)
  C acc[KPT];
  unsigned kq[KPT];
#pragma unroll
  for (int u = 0; u < KPT; ++u) {
    const int q = tid + TPB * u;
    kq[u] = q < l ? (unsigned)idx[order[q]] : 0u;  // idx < N (checked before the launch)
    acc[u] = vzero<C>();
  }
  // slot u's (W_N^k, W_N^{B k}), from the table k_sketch_order laid out in
  // slot order (a coalesced read).  The empty asm makes k and the slot
  // opaque inside the block loop, so the reads that depend on them stay
  // there (hoisted, they would hold 4 KPT more registers through the loop).
  const C* stp = kept_steps<C>(order, l);
  auto kept = [&](int u) -> unsigned {
    unsigned k = kq[u];
    asm volatile("" : "+v"(k));
    return k;
  };
  auto steps = [&](int u, C& st, C& sb) {
    int q = tid + TPB * u;
    asm volatile("" : "+v"(q));
    q = q < l ? q : 0;
    st = stp[2 * q];
    sb = stp[2 * q + 1];
  };

  // the next block's entries of A are loaded into registers before the
  // outer sum and used after it; A is read once, as a stream (non-temporal:
  // it does not push the phase and twiddle tables, which every row reads,
  // out of the cache).  The phases are read when the block is formed.
  // Columns n1 >= N1 of a last, partial block are zero (their transforms
  // add nothing to the outer sum).
  V pa[16];
  auto load = [&](int c0) {
    const bool col = c0 + bb < N1;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t j = (int64_t)(c0 + bb) + (int64_t)N1 * (jj + r * LR);
      pa[r] = (col && j < n) ? ld_stream(row + j) : V{};
    }
  };
  // blocks in decreasing order: the group's sum
  //   sum_g W_N^{(cbeg + g B) k} H_g = W_N^{cbeg k} sum_g (W_N^{B k})^g H_g
  // (H_g = the block's share with its columns counted from c0) is a
  // polynomial in W_N^{B k}, evaluated by Horner's rule across the blocks
  const int cbeg = bk.x * G * B;
  load(cbeg + (G - 1) * B);
  for (int g = G - 1; g >= 0; --g) {
    const int c0 = cbeg + g * B;
    {
      C v[16];
      const bool col = c0 + bb < N1;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t j = (int64_t)(c0 + bb) + (int64_t)N1 * (jj + r * LR);
        const D dd = (col && j < n) ? dp[j] : D{};
        if constexpr (VT<V>::cplx) v[r] = vcmul(vconv<C>(pa[r]), vmake<C>(dd.re, dd.im));  // conj(a) d
        else v[r] = C{(R)pa[r] * (R)dd, (R)0};
      }
      dft16(v);
      C* buf = sm + bb * Lp;
#pragma unroll
      for (int r = 0; r < 16; ++r) buf[lpad(jj * 16 + r)] = v[out_slot<16>(r)];
    }
    __syncthreads();
    {
      C* buf = sm + fb * Lp;
      int Ns = 16;
      for (int s = 1; s < pl2.nst; ++s) {
        const int Rd = pl2.radix[s];
        if (Rd == 16) fft_stage<16>(buf, N2, Ns, LR, tl, twst, twm);
        else if (Rd == 8) fft_stage<8>(buf, N2, Ns, LR, tl, twst, twm);
        else if (Rd == 4) fft_stage<4>(buf, N2, Ns, LR, tl, twst, twm);
        else fft_stage<2>(buf, N2, Ns, LR, tl, twst, twm);
        Ns *= Rd;
      }
    }
    // Z of the block is in LDS (the last stage ends with a barrier); the
    // next block's loads fly during the outer sum
    if (g > 0) load(c0 - B);
    // two kept outputs at a time (two independent chains interleave; the
    // scheduling barrier keeps the next pair's LDS reads from being hoisted
    // into this one's registers).  The block's share
    //   H_g = sum_b (W_N^k)^b Z_{c0+b}
    // by Horner's rule too (one complex multiply-add per column), then
    //   acc = acc W_N^{B k} + H_g
#pragma unroll
    for (int u = 0; u < KPT; u += 2) {
      const unsigned k0 = kept(u), k1 = kept(u + 1);
      C st0, sb0, st1, sb1;
      steps(u, st0, sb0);
      steps(u + 1, st1, sb1);
      const C* zp0 = sm + lpad((int)(k0 & (unsigned)(N2 - 1)));
      const C* zp1 = sm + lpad((int)(k1 & (unsigned)(N2 - 1)));
      C h0 = lds_c(zp0 + (B - 1) * Lp), h1 = lds_c(zp1 + (B - 1) * Lp);
#pragma unroll
      for (int b = B - 2; b >= 0; --b) {
        h0 = vfma(h0, st0, lds_c(zp0 + b * Lp));
        h1 = vfma(h1, st1, lds_c(zp1 + b * Lp));
      }
      acc[u] = vfma(acc[u], sb0, h0);
      acc[u + 1] = vfma(acc[u + 1], sb1, h1);
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < KPT; ++u) {
    const int q = tid + TPB * u;
    if (q < l) {
      const int64_t s = order[q];
      C a = acc[u];
      if (cbeg > 0) a = vmul(a, tw[(uint64_t)cbeg * kq[u] % Ntot]);  // W_N^{cbeg k}
      if (bk.gx == 1) S[s + i * lds] = out_value<V, C>(a, scale);
      else P[((int64_t)bk.x * rows + bk.y) * l + s] = a;
    }
  }
}
template <typename V, typename C, int B, int KPT, int TPB = 256>
__global__ void __launch_bounds__(TPB, TPB == 256 ? 2 : 1) k_sketch_pruned(
    const V* __restrict__ A, int64_t lda, int64_t row0, int64_t rows, int64_t n, int N1, int G, FftPlan pl2,
    const void* __restrict__ dv, const int32_t* __restrict__ idx, const int32_t* __restrict__ order, int64_t l,
    const C* __restrict__ tw, V* __restrict__ S, int64_t lds, C* __restrict__ P, typename VT<C>::real scale) {
  k_sketch_pruned_body<V, C, B, KPT, TPB>(bk_hw(), A, lda, row0, rows, n, N1, G, pl2, dv, idx, order, l, tw, S, lds, P,
                                          scale);
}

// order[0 .. l) = a permutation of 0 .. l that groups the kept outputs by
// idx[s] mod N2 (counting sort on the residue; the order inside a group is
// whatever the LDS atomics give, which changes no result), and, when tw is
// given, beside it the kept-output table in the same order: (W_N^k,
// W_N^{B k}) with k = idx[s] (k_sketch_steps fills it over many workgroups).
// One workgroup of 1024 threads; N2 <= kOrderMaxN2 (the counts live in LDS;
// their exclusive prefix sum runs in parallel: each thread sums a run of
// N2 / 1024 counts, the run totals are scanned across the workgroup, then
// each run is filled).
constexpr int kOrderMaxN2 = 16384;
template <typename C>
__device__ __forceinline__ void k_sketch_order_body(const int32_t* __restrict__ idx, int64_t l, int N2, int64_t N,
                                                    int B, const C* __restrict__ tw, int32_t* __restrict__ order) {
  __shared__ int cnt[kOrderMaxN2];
  __shared__ int tot[1024];
  const int tid = threadIdx.x;
  for (int r = tid; r < N2; r += 1024) cnt[r] = 0;
  __syncthreads();
  for (int64_t s = tid; s < l; s += 1024) atomicAdd(&cnt[idx[s] & (N2 - 1)], 1);
  __syncthreads();
  const int per = (N2 + 1023) / 1024, r0 = tid * per;
  int run = 0;
  for (int r = r0; r < r0 + per && r < N2; ++r) run += cnt[r];
  tot[tid] = run;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive scan of the run totals
    const int v = tid >= d ? tot[tid - d] : 0;
    __syncthreads();
    tot[tid] += v;
    __syncthreads();
  }
  int base = tot[tid] - run;  // exclusive
  for (int r = r0; r < r0 + per && r < N2; ++r) {
    const int c = cnt[r];
    cnt[r] = base;
    base += c;
  }
  __syncthreads();
  C* steps = const_cast<C*>(kept_steps<C>(order, l));
  for (int64_t s = tid; s < l; s += 1024) {
    const int64_t k = idx[s];
    const int pos = atomicAdd(&cnt[k & (N2 - 1)], 1);
    order[pos] = (int32_t)s;
    if (tw != nullptr) {
      steps[2 * (int64_t)pos] = tw[k];
      steps[2 * (int64_t)pos + 1] = tw[(int64_t)B * k % N];
    }
  }
}
// the kept-output table from the order: slot q gets (W_N^k, W_N^{B k}),
// k = idx[order[q]].  grid ceil(l / 256), 256 threads.
template <typename C>
__global__ void __launch_bounds__(256) k_sketch_steps(const int32_t* __restrict__ idx, int64_t l, int64_t N, int B,
                                                      const C* __restrict__ tw, int32_t* __restrict__ order) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= l) return;
  const int64_t k = idx[order[q]];
  C* steps = const_cast<C*>(kept_steps<C>(order, l));
  steps[2 * q] = tw[k];
  steps[2 * q + 1] = tw[(int64_t)B * k % N];
}
template <typename C>
__global__ void __launch_bounds__(1024) k_sketch_order(const int32_t* __restrict__ idx, int64_t l, int N2, int64_t N,
                                                       int B, const C* __restrict__ tw, int32_t* __restrict__ order) {
  k_sketch_order_body<C>(idx, l, N2, N, B, tw, order);
}

// S[s + i lds] = scale * sum over the ng column groups of P[g][i - row0][s]
// grid (ceil(l / 256), rows)
template <typename V, typename C>
__global__ void __launch_bounds__(256) k_sketch_fold(const C* __restrict__ P, int ng, int64_t rows, int64_t l,
                                                     int64_t row0, V* __restrict__ S, int64_t lds,
                                                     typename VT<C>::real scale) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (s >= l) return;
  C a = P[r * l + s];
  for (int g = 1; g < ng; ++g) a = vadd(a, P[((int64_t)g * rows + r) * l + s]);
  S[s + (row0 + r) * lds] = out_value<V, C>(a, scale);
}

// ------------------------------ helpers -------------------------------------
// inv[k] = position of k in idx, or -1; also flags invalid idx (out of range
// or not strictly increasing) in *bad.  Writes stay inside inv[0, N).
__device__ __forceinline__ void k_fill_i32_body(const Bk bk, int32_t* p, int64_t count, int32_t v) {
  const int64_t t = (int64_t)bk.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = v;
}
__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t v) {
  k_fill_i32_body(bk_hw(), p, count, v);
}

__device__ __forceinline__ void k_inverse_map_body(const Bk bk, const int32_t* __restrict__ idx, int64_t l, int64_t N, int32_t* __restrict__ inv,
                              int32_t* __restrict__ bad) {
  const int64_t k = (int64_t)bk.x * blockDim.x + threadIdx.x;
  if (k >= l) return;
  const int32_t v = idx[k];
  bool ok = v >= 0 && (int64_t)v < N;
  if (k + 1 < l && !(idx[k + 1] > v)) ok = false;
  if (ok) inv[v] = (int32_t)k;
  else atomicOr(bad, 1);
}
__global__ void k_inverse_map(const int32_t* __restrict__ idx, int64_t l, int64_t N, int32_t* __restrict__ inv,
                              int32_t* __restrict__ bad) {
  k_inverse_map_body(bk_hw(), idx, l, N, inv, bad);
}

// ------------------------------ launchers -----------------------------------
FftPlan make_plan(int L) {
  FftPlan p{};
  p.L = L;
  int k = 0;
  while ((1 << k) < L) ++k;
  p.nst = 0;
  while (k >= 4) { p.radix[p.nst++] = 16; k -= 4; }
  if (k > 0) p.radix[p.nst++] = 1 << k;
  return p;
}


// Per-workgroup LDS limit of the current device (bytes).
static int lds_limit() {
  // queried once (thread-safe static initialisation)
  static const int v = [] {
    int dev = 0, x = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&x, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && x > 0)
      return x;
    return 65536;
  }();
  return v;
}

template <typename C> static int max_lds_fft_len() {
  int L = kFftMaxLds;
  while (L > 16 && (int64_t)lds_stride(L) * (int64_t)sizeof(C) > lds_limit()) L >>= 1;
  return L;
}

template <typename K> static void allow_lds(K* kern, size_t bytes) {
  if (bytes > 48 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

// transforms per workgroup: up to 4096 elements (256 threads x 16) within LDS
template <typename C> static int fft_batch(int L, int elems = 4096) {
  int B = elems / L;
  if (B > 256) B = 256;  // L < 16: one thread per transform
  if (B < 1) B = 1;
  while (B > 1 && (int64_t)B * lds_stride(L) * (int64_t)sizeof(C) > lds_limit()) B >>= 1;
  return B;
}

// Column groups per row of the pruned four-step for B columns per block and
// ng groups asked for (clamped to 1 .. N1 / B), or 0 where it does not apply:
// more kept outputs than accumulators fit (eight per thread in FP64,
// thirty-two in FP32, times the workgroup's threads), N not a multiple of
// N2 = 16 tpb / B, or a block larger than the LDS limit.
// workgroup widths of the kept-outputs-only form: 256 threads, and a wide
// form of 512 threads (8192 elements, so that N2 reaches 2048 at B = 4; two
// workgroups to a CU in single precision, one in double).  1024 threads
// would cap a thread at 128 registers and spill.
template <typename C> static constexpr int pruned_wide_tpb() { return 512; }

template <typename C> static size_t pruned_smem(int B, int tpb) {
  const int N2 = tpb * 16 / B;
  const int64_t cols = (int64_t)B * lds_stride(N2) * (int64_t)sizeof(C);
  const int64_t with_tw = cols + (int64_t)N2 * (int64_t)sizeof(C);
  bool twl;
  if (tpb == 256) twl = B >= 8;
  else twl = with_tw <= 80 * 1024 || (cols > 80 * 1024 && with_tw <= 160 * 1024);
  return (size_t)(twl ? with_tw : cols);
}

template <typename C> static int pruned_groups(int64_t N, int64_t l, int B, int ng, int tpb = 256) {
  if (tpb != 256 && tpb != pruned_wide_tpb<C>()) return 0;
  const int64_t kmax = std::is_same<C, cf>::value ? 32 : 8;  // accumulators per thread
  if (!(B == 16 || B == 8 || B == 4) || l < 1 || l > kmax * tpb) return 0;
  const int64_t N2 = (int64_t)tpb * 16 / B;
  if (N2 > kOrderMaxN2 || N <= N2 || N % N2) return 0;
  if ((int64_t)pruned_smem<C>(B, tpb) > lds_limit()) return 0;
  const int64_t nb = ceil_div(N / N2, B);  // blocks per row (the last one partial when B does not divide N1)
  if (nb < 1) return 0;
  int g = ng < 1 ? 1 : ng;
  while (g > 1 && (nb % g || g > nb)) g >>= 1;
  return g;
}

template <typename V, typename C, int B, int KPT, int TPB>
static void pruned_go(dim3 grid, size_t smb, hipStream_t st, const V* A, int64_t lda, int64_t row0, int64_t rows,
                      int64_t n, int N1, int G, FftPlan pl2, const void* d, const int32_t* idx, const int32_t* order,
                      int64_t l, const C* tw, V* S, int64_t lds, C* P, typename VT<C>::real scale) {
  allow_lds(k_sketch_pruned<V, C, B, KPT, TPB>, smb);
  hipLaunchKernelGGL((k_sketch_pruned<V, C, B, KPT, TPB>), grid, dim3(TPB), smb, st, A, lda, row0, rows, n, N1, G, pl2,
                     d, idx, order, l, tw, S, lds, P, scale);
}

template <typename V, typename C, int B, int TPB>
static void pruned_launch(int kpt, dim3 grid, size_t smb, hipStream_t st, const V* A, int64_t lda, int64_t row0,
                          int64_t rows, int64_t n, int N1, int G, FftPlan pl2, const void* d, const int32_t* idx,
                          const int32_t* order, int64_t l, const C* tw, V* S, int64_t lds, C* P,
                          typename VT<C>::real scale) {
  if (kpt == 2)
    pruned_go<V, C, B, 2, TPB>(grid, smb, st, A, lda, row0, rows, n, N1, G, pl2, d, idx, order, l, tw, S, lds, P, scale);
  else if (kpt == 4)
    pruned_go<V, C, B, 4, TPB>(grid, smb, st, A, lda, row0, rows, n, N1, G, pl2, d, idx, order, l, tw, S, lds, P, scale);
  else if (kpt == 8)
    pruned_go<V, C, B, 8, TPB>(grid, smb, st, A, lda, row0, rows, n, N1, G, pl2, d, idx, order, l, tw, S, lds, P, scale);
  else if constexpr (std::is_same<C, cf>::value) {
    // FP32 accumulators: up to 32 kept outputs per thread
    if (kpt == 16)
      pruned_go<V, C, B, 16, TPB>(grid, smb, st, A, lda, row0, rows, n, N1, G, pl2, d, idx, order, l, tw, S, lds, P,
                                  scale);
    else
      pruned_go<V, C, B, 32, TPB>(grid, smb, st, A, lda, row0, rows, n, N1, G, pl2, d, idx, order, l, tw, S, lds, P,
                                  scale);
  }
}

template <typename V, typename C, int B>
static void pruned_launch_tpb(int tpb, int kpt, dim3 grid, size_t smb, hipStream_t st, const V* A, int64_t lda,
                              int64_t row0, int64_t rows, int64_t n, int N1, int G, FftPlan pl2, const void* d,
                              const int32_t* idx, const int32_t* order, int64_t l, const C* tw, V* S, int64_t lds,
                              C* P, typename VT<C>::real scale) {
  if (tpb == 256)
    pruned_launch<V, C, B, 256>(kpt, grid, smb, st, A, lda, row0, rows, n, N1, G, pl2, d, idx, order, l, tw, S, lds, P,
                                scale);
  else
    pruned_launch<V, C, B, pruned_wide_tpb<C>()>(kpt, grid, smb, st, A, lda, row0, rows, n, N1, G, pl2, d, idx, order,
                                                 l, tw, S, lds, P, scale);
}

template <typename V, typename C>
static hipError_t sketch_pruned_impl(const SketchArgs& a, hipStream_t st) {
  const int N = (int)a.N;
  const int B = a.pruned_b;
  const int tpb = a.pruned_tpb > 0 ? a.pruned_tpb : 256;
  const int ng = pruned_groups<C>(a.N, a.l, B, a.pruned_ng, tpb);
  if (ng < 1) return hipErrorInvalidValue;
  const int N2 = tpb * 16 / B, N1 = N / N2;
  const int G = (int)ceil_div(N1, B) / ng;
  const int64_t per_thread = ceil_div(a.l, tpb);
  const int kpt = per_thread <= 2 ? 2 : (per_thread <= 4 ? 4 : (per_thread <= 8 ? 8 : (per_thread <= 16 ? 16 : 32)));
  const FftPlan pl2 = make_plan(N2);
  using R = typename VT<C>::real;
  const R scale = (R)(1.0 / sqrt((double)N));
  const C* tw = reinterpret_cast<const C*>(a.twiddle);
  const V* A = reinterpret_cast<const V*>(a.A);
  V* S = reinterpret_cast<V*>(a.S);
  C* P = reinterpret_cast<C*>(a.work);
  const size_t smb = pruned_smem<C>(B, tpb);
  // one group per row: no partial sums, every row in one launch
  const int64_t per = ng == 1 ? a.m : a.chunk_rows;
  if (per < 1 || (ng > 1 && P == nullptr) || a.order == nullptr) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sketch_order<C>), dim3(1), dim3(1024), 0, st, a.idx, a.l, N2, a.N, B, (const C*)nullptr,
                     a.order);
  hipLaunchKernelGGL((k_sketch_steps<C>), dim3((unsigned)ceil_div(a.l, 256)), dim3(256), 0, st, a.idx, a.l, a.N, B, tw,
                     a.order);
  for (int64_t r0 = 0; r0 < a.m; r0 += per) {
    const int64_t rows = (a.m - r0) < per ? (a.m - r0) : per;
    const dim3 grid((unsigned)ng, (unsigned)rows);
    if (B == 16)
      pruned_launch_tpb<V, C, 16>(tpb, kpt, grid, smb, st, A, a.lda, r0, rows, a.n, N1, G, pl2, a.d, a.idx, a.order, a.l, tw, S, a.lds,
                              P, scale);
    else if (B == 8)
      pruned_launch_tpb<V, C, 8>(tpb, kpt, grid, smb, st, A, a.lda, r0, rows, a.n, N1, G, pl2, a.d, a.idx, a.order, a.l, tw, S, a.lds,
                             P, scale);
    else
      pruned_launch_tpb<V, C, 4>(tpb, kpt, grid, smb, st, A, a.lda, r0, rows, a.n, N1, G, pl2, a.d, a.idx, a.order, a.l, tw, S, a.lds,
                             P, scale);
    if (ng > 1)
      hipLaunchKernelGGL((k_sketch_fold<V, C>), dim3((unsigned)ceil_div(a.l, 256), (unsigned)rows), dim3(256), 0, st,
                         P, ng, rows, a.l, r0, S, a.lds, scale);
  }
  return hipGetLastError();
}

template <typename V, typename C>
static hipError_t sketch_impl(const SketchArgs& a, hipStream_t st) {
  const int N = (int)a.N;
  const C* tw = reinterpret_cast<const C*>(a.twiddle);
  using R = typename VT<C>::real;
  const R scale = (R)(1.0 / sqrt((double)N));
  const V* A = reinterpret_cast<const V*>(a.A);
  V* S = reinterpret_cast<V*>(a.S);
  const int Lmax = max_lds_fft_len<C>();
  const bool p2 = (N & (N - 1)) == 0;
  // a length that is not a power of two runs only in the kept-outputs-only
  // form (the radix plans below cover powers of two only)
  if (!p2 && a.pruned_b <= 0) return hipErrorInvalidValue;
  if (p2 && N <= Lmax) {
    FftPlan pl = make_plan(N);
    const int B = fft_batch<C>(N);
    const size_t sm = (size_t)B * lds_stride(N) * sizeof(C);
    allow_lds(k_sketch_small<V, C>, sm);
    dim3 grid((unsigned)ceil_div(a.m, B));
    hipLaunchKernelGGL((k_sketch_small<V, C>), grid, dim3(256), sm, st, A, a.lda, a.m, a.n, pl, B, a.d, a.idx,
                       a.l, S, a.lds, tw, scale);
    return hipGetLastError();
  }
  if (a.pruned_b > 0) return sketch_pruned_impl<V, C>(a, st);
  // four-step: N = N1 * N2, N1 >= N2, both transformed whole in LDS; split
  // s halves N2 s times (fewer for shapes where N1 would outgrow LDS)
  int k = 0;
  while ((1 << k) < N) ++k;
  const int N2_0 = 1 << (k / 2), N1_0 = N >> (k / 2);
  int split = a.split < 0 ? 0 : (a.split > 2 ? 2 : a.split);
  while (split > 0 && ((N1_0 << split) > Lmax || (N2_0 >> split) < 16)) --split;
  const int N2 = N2_0 >> split, N1 = N1_0 << split;
  if (N1 > Lmax) return hipErrorInvalidValue;
  const C* twc = tw + N + (split == 0 ? 0 : split == 1 ? N1_0 : 3 * N1_0);
  FftPlan pl1 = make_plan(N1), pl2 = make_plan(N2);
  // fewer elements per workgroup (half the threads idle in the transform,
  // all of them load) halve the LDS footprint and double the workgroups
  // resident per CU
  const int elems = a.wg_elems == 2048 ? 2048 : 4096;
  const int Bc = fft_batch<C>(N2, elems);  // columns per workgroup, pass 1
  const int Br = fft_batch<C>(N1, elems);  // rows of the intermediate per workgroup, pass 2
  const size_t smc = (size_t)Bc * lds_stride(N2) * sizeof(C);
  const size_t smr = (size_t)Br * lds_stride(N1) * sizeof(C);
  allow_lds(k_sketch_cols<V, C>, smc);
  allow_lds(k_sketch_rows<V, C>, smr);
  C* Y = reinterpret_cast<C*>(a.work);
  for (int64_t r0 = 0; r0 < a.m; r0 += a.chunk_rows) {
    const int64_t rows = (a.m - r0) < a.chunk_rows ? (a.m - r0) : a.chunk_rows;
    dim3 g1((unsigned)(N1 / Bc), (unsigned)rows);
    hipLaunchKernelGGL((k_sketch_cols<V, C>), g1, dim3(256), smc, st, A, a.lda, r0, a.m, a.n, N1, pl2, Bc, a.d, Y,
                       tw, twc);
    dim3 g2((unsigned)(N2 / Br), (unsigned)rows);
    hipLaunchKernelGGL((k_sketch_rows<V, C>), g2, dim3(256), smr, st, Y, r0, a.m, N2, pl1, Br, a.inv, S, a.lds, twc,
                       scale);
  }
  return hipGetLastError();
}

int sketch_pruned_groups(int dtype, int64_t N, int64_t l, int B, int ng, int tpb) {
  const bool sp = dtype == 1 || dtype == 3;
  const bool p2 = N > 0 && (N & (N - 1)) == 0;
  // a power of two that fits one workgroup's LDS takes the whole-row transform
  if (p2 && N <= (sp ? max_lds_fft_len<cf>() : max_lds_fft_len<cd>())) return 0;
  return sp ? pruned_groups<cf>(N, l, B, ng, tpb) : pruned_groups<cd>(N, l, B, ng, tpb);
}

int64_t sketch_order_bytes(int64_t l, bool single) { return ((4 * l + 255) & ~(int64_t)255) + 2 * l * (single ? 8 : 16); }

int sketch_pruned_wide_tpb(int dtype) { return (dtype == 1 || dtype == 3) ? pruned_wide_tpb<cf>() : pruned_wide_tpb<cd>(); }

int sketch_max_log2n(int dtype) {
  const int L = (dtype == 1 || dtype == 3) ? max_lds_fft_len<cf>() : max_lds_fft_len<cd>();
  int k = 0;
  while ((1 << k) < L) ++k;
  return 2 * k;
}

// Twiddle table: W_N^k = exp(-2 pi i k / N) for k < N, then the compact
// tables W_L^k (k < L) for L = N1, 2 N1, 4 N1 where L <= N, N1 = N / 2^floor(
// log2(N) / 2) (the four-step splits).  cos and sin of pi (-2k / L), an exact
// argument, in FP64, rounded once to the table's precision.
template <typename C>
__global__ void __launch_bounds__(256) k_twiddles(int64_t N, int64_t N1, int64_t total, C* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= total) return;
  int64_t k = t, L = N;
  if (t >= N) {
    int64_t off = N;
    for (int s = 0; s < 3; ++s) {
      const int64_t Ls = N1 << s;
      if (t < off + Ls) {
        k = t - off;
        L = Ls;
        break;
      }
      off += Ls;
    }
  }
  double sn, cs;
  sincospi(-2.0 * (double)k / (double)L, &sn, &cs);
  out[t] = vmake<C>(cs, sn);
}

static int64_t twiddle_n1(int64_t N) {
  int lg = 0;
  while (((int64_t)1 << lg) < N) ++lg;
  return N >> (lg / 2);
}

int64_t twiddle_entries(int64_t N) {
  const int64_t N1 = twiddle_n1(N);
  int64_t total = N;
  for (int s = 0; s < 3; ++s)
    if ((N1 << s) <= N) total += N1 << s;
  return total;
}

hipError_t launch_twiddles(bool single, int64_t N, void* out, hipStream_t st) {
  const int64_t total = twiddle_entries(N);
  const dim3 grid((unsigned)ceil_div(total, 256));
  if (single)
    hipLaunchKernelGGL((k_twiddles<cf>), grid, dim3(256), 0, st, N, twiddle_n1(N), total, reinterpret_cast<cf*>(out));
  else
    hipLaunchKernelGGL((k_twiddles<cd>), grid, dim3(256), 0, st, N, twiddle_n1(N), total, reinterpret_cast<cd*>(out));
  return hipGetLastError();
}

hipError_t launch_inverse_map(const int32_t* idx, int64_t l, int64_t N, int32_t* inv, int32_t* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, st, inv, N, -1);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, st, bad, 1, 0);
  hipLaunchKernelGGL(k_inverse_map, dim3((unsigned)ceil_div(l, 256)), dim3(256), 0, st, idx, l, N, inv, bad);
  return hipGetLastError();
}

int64_t sketch_work_elems(int64_t N, int64_t chunk_rows) {
  return N * chunk_rows;
}

hipError_t launch_sketch(int dtype, const SketchArgs& a, hipStream_t st) {
  switch (dtype) {
    case 0: return sketch_impl<cd, cd>(a, st);
    case 1: return sketch_impl<cf, cf>(a, st);
    case 2: return sketch_impl<double, cd>(a, st);
    case 3: return sketch_impl<float, cf>(a, st);
  }
  return hipErrorInvalidValue;
}

// ------------------------------ batched systems -------------------------------
namespace {

template <typename V, typename C>
__global__ void __launch_bounds__(256) kb_sketch_small(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                       int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  using R = typename VT<C>::real;
  k_sketch_small_body<V, C>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<const V*>(s.Ab),
                            s.ldab, s.m, s.n, s.pl_a, s.fft_ba, s.d, s.idx, s.l, reinterpret_cast<V*>(s.S), s.l,
                            reinterpret_cast<const C*>(s.tw), (R)(1.0 / sqrt((double)s.N)));
}

template <typename V, typename C>
__global__ void __launch_bounds__(256) kb_sketch_cols(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                      int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_sketch_cols_body<V, C>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<const V*>(s.Ab),
                           s.ldab, 0, s.m, s.n, s.N1, s.pl_b, s.fft_bb, s.d, reinterpret_cast<C*>(s.Y),
                           reinterpret_cast<const C*>(s.tw), reinterpret_cast<const C*>(s.tw) + s.N);
}

template <typename V, typename C>
__global__ void __launch_bounds__(256) kb_sketch_rows(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                      int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  using R = typename VT<C>::real;
  k_sketch_rows_body<V, C>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<const C*>(s.Y), 0,
                           s.m, s.N2, s.pl_a, s.fft_ba, s.inv, reinterpret_cast<V*>(s.S), s.l,
                           reinterpret_cast<const C*>(s.tw) + s.N, (R)(1.0 / sqrt((double)s.N)));
}

// kept-outputs-only four-step (B = 16, one column group per row): one
// workgroup per row of a system; KPT = the system's accumulator class
template <typename V, typename C, int KPT>
__global__ void __launch_bounds__(256, 2) kb_sketch_pruned(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                           int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  using R = typename VT<C>::real;
  const Bk bk = bgrid_local(grid[i], (int)blockIdx.x - grid[i].start);
  const R scale = (R)(1.0 / sqrt((double)s.N));
  k_sketch_pruned_body<V, C, 16, KPT, 256>(bk, reinterpret_cast<const V*>(s.Ab), s.ldab, 0, s.m, s.n, s.N1,
                                           (s.N1 + 15) / 16, s.pl_b, s.d, s.idx, s.order, s.l,
                                           reinterpret_cast<const C*>(s.tw), reinterpret_cast<V*>(s.S), s.l, nullptr,
                                           scale);
}

template <typename C>
__global__ void __launch_bounds__(1024) kb_sketch_order(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                        int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_sketch_order_body<C>(s.idx, s.l, s.N2, s.N, 16, reinterpret_cast<const C*>(s.tw), s.order);
}

__global__ void kb_fill_inv(const BSys* __restrict__ sys, const BGrid* __restrict__ grid, int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_fill_i32_body(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), s.inv, s.N, -1);
}

__global__ void kb_inverse_map(const BSys* __restrict__ sys, const BGrid* __restrict__ grid, int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_inverse_map_body(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), s.idx, s.l, s.N, s.inv, s.flags);
}

template <typename C> void plan_sketch_t(BSys& s, BGrid& small, BGrid& cols, BGrid& rows, BGrid& pruned, size_t& ls,
                                         size_t& lc, size_t& lr, size_t& lp) {
  const int N = (int)s.N;
  small = BGrid{0, 0, 1, 1};
  cols = BGrid{0, 0, 1, 1};
  rows = BGrid{0, 0, 1, 1};
  pruned = BGrid{0, 0, 1, 1};
  ls = lc = lr = lp = 0;
  s.sk_kpt = 0;
  const bool p2 = (N & (N - 1)) == 0;
  if (p2 && N <= max_lds_fft_len<C>()) {
    s.pl_a = make_plan(N);
    s.fft_ba = fft_batch<C>(N);
    s.N1 = N;
    s.N2 = 1;
    small.gx = (int)ceil_div(s.m, s.fft_ba);
    ls = (size_t)s.fft_ba * lds_stride(N) * sizeof(C);
    return;
  }
  if (s.l <= 2048 && pruned_groups<C>(N, s.l, 16, 1) > 0) {
    // kept outputs only: N2 = 256, one workgroup per row
    s.N2 = 256;
    s.N1 = N / 256;
    s.pl_b = make_plan(256);
    s.sk_kpt = s.l <= 512 ? 2 : (s.l <= 1024 ? 4 : 8);
    pruned = BGrid{0, 1, (int)s.m, 1};
    lp = ((size_t)16 * lds_stride(256) + 256) * sizeof(C);
    return;
  }
  int k = 0;
  while ((1 << k) < N) ++k;
  s.N2 = 1 << (k / 2);
  s.N1 = N >> (k / 2);
  s.pl_a = make_plan(s.N1);
  s.pl_b = make_plan(s.N2);
  s.fft_bb = fft_batch<C>(s.N2);
  s.fft_ba = fft_batch<C>(s.N1);
  cols.gx = s.N1 / s.fft_bb;
  cols.gy = (int)s.m;
  rows.gx = s.N2 / s.fft_ba;
  rows.gy = (int)s.m;
  lc = (size_t)s.fft_bb * lds_stride(s.N2) * sizeof(C);
  lr = (size_t)s.fft_ba * lds_stride(s.N1) * sizeof(C);
}

template <typename V, typename C>
hipError_t b_sketch_t(const BLaunch& sm, const BLaunch& co, const BLaunch& ro, const BLaunch& ord, const BLaunch* pr,
                      size_t ls, size_t lc, size_t lr, size_t lp, hipStream_t st) {
  if (ord.total > 0) {
    hipLaunchKernelGGL((kb_sketch_order<C>), dim3((unsigned)ord.total), dim3(1024), 0, st, ord.sys, ord.grid,
                       ord.nsys);
    if (pr[0].total > 0) {
      allow_lds(kb_sketch_pruned<V, C, 2>, lp);
      hipLaunchKernelGGL((kb_sketch_pruned<V, C, 2>), dim3((unsigned)pr[0].total), dim3(256), lp, st, pr[0].sys,
                         pr[0].grid, pr[0].nsys);
    }
    if (pr[1].total > 0) {
      allow_lds(kb_sketch_pruned<V, C, 4>, lp);
      hipLaunchKernelGGL((kb_sketch_pruned<V, C, 4>), dim3((unsigned)pr[1].total), dim3(256), lp, st, pr[1].sys,
                         pr[1].grid, pr[1].nsys);
    }
    if (pr[2].total > 0) {
      allow_lds(kb_sketch_pruned<V, C, 8>, lp);
      hipLaunchKernelGGL((kb_sketch_pruned<V, C, 8>), dim3((unsigned)pr[2].total), dim3(256), lp, st, pr[2].sys,
                         pr[2].grid, pr[2].nsys);
    }
  }
  if (sm.total > 0) {
    allow_lds(kb_sketch_small<V, C>, ls);
    hipLaunchKernelGGL((kb_sketch_small<V, C>), dim3((unsigned)sm.total), dim3(256), ls, st, sm.sys, sm.grid,
                       sm.nsys);
  }
  if (co.total > 0) {
    allow_lds(kb_sketch_cols<V, C>, lc);
    allow_lds(kb_sketch_rows<V, C>, lr);
    hipLaunchKernelGGL((kb_sketch_cols<V, C>), dim3((unsigned)co.total), dim3(256), lc, st, co.sys, co.grid,
                       co.nsys);
    hipLaunchKernelGGL((kb_sketch_rows<V, C>), dim3((unsigned)ro.total), dim3(256), lr, st, ro.sys, ro.grid,
                       ro.nsys);
  }
  return hipGetLastError();
}

}  // namespace

void b_plan_sketch(int dtype, BSys& s, BGrid& small, BGrid& cols, BGrid& rows, BGrid& pruned, size_t& ls, size_t& lc,
                   size_t& lr, size_t& lp) {
  if (dtype == 1 || dtype == 3) plan_sketch_t<cf>(s, small, cols, rows, pruned, ls, lc, lr, lp);
  else plan_sketch_t<cd>(s, small, cols, rows, pruned, ls, lc, lr, lp);
}

int64_t b_sketch_work_elems(int dtype, int64_t m, int64_t N, int64_t l) {
  const int L = (dtype == 1 || dtype == 3) ? max_lds_fft_len<cf>() : max_lds_fft_len<cd>();
  const bool p2 = (N & (N - 1)) == 0;
  if ((p2 && N <= L) || (l <= 2048 && sketch_pruned_groups(dtype, N, l, 16, 1) > 0)) return 0;
  return m * N;
}

hipError_t launch_b_prep(const BLaunch& fill, const BLaunch& map, hipStream_t st) {
  hipLaunchKernelGGL(kb_fill_inv, dim3((unsigned)fill.total), dim3(256), 0, st, fill.sys, fill.grid, fill.nsys);
  hipLaunchKernelGGL(kb_inverse_map, dim3((unsigned)map.total), dim3(256), 0, st, map.sys, map.grid, map.nsys);
  return hipGetLastError();
}

hipError_t launch_b_sketch(int dtype, const BLaunch& small, const BLaunch& cols, const BLaunch& rows,
                           const BLaunch& order, const BLaunch* pruned, size_t ls, size_t lc, size_t lr, size_t lp,
                           hipStream_t st) {
  switch (dtype) {
    case 0: return b_sketch_t<cd, cd>(small, cols, rows, order, pruned, ls, lc, lr, lp, st);
    case 1: return b_sketch_t<cf, cf>(small, cols, rows, order, pruned, ls, lc, lr, lp, st);
    case 2: return b_sketch_t<double, cd>(small, cols, rows, order, pruned, ls, lc, lr, lp, st);
    case 3: return b_sketch_t<float, cf>(small, cols, rows, order, pruned, ls, lc, lr, lp, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace mn
