// The FP64 refinement residual's product q = A (A* y) in one pass over a
// column-major copy of A, with compensated (double-double) sums, for m up to
// 2048; also x = A* y, the same column sums, as a by-product.
//
// The two-pass form (an adjoint pass, then a forward pass) reads A twice per
// refinement step.  Here a column group of WPC waves holds whole columns of
// the copy (wave w: rows w 64 RPT .. (w + 1) 64 RPT - 1, one entry per lane
// and load), forms the column sum w_c = sum_r conj(A_rc) y_r in
// double-double (TwoProd by FMA, TwoSum; Ogita, Rump and Oishi 2005), reduces
// it over the wave (lane 0's value, the same for every lane after the
// broadcast) and over the group's waves in wave order through LDS, rounds it
// once to FP64 -- exactly what the two-pass form stores between its passes --
// and adds A_rc w_c to the rows' double-double accumulators.  Each workgroup
// leaves (hi, lo) partials of q; a fold adds them in a fixed order and
// rounds once.  The column sums are written as x = A* y when asked for.
// Rows m .. ldt - 1 of the copy are not read.
#include "common.hpp"
#include "kernels.hpp"

namespace mn {

namespace {

struct dd2 {
  double hi, lo;
};

__device__ inline void d2_add(dd2& a, double x) {
#pragma clang fp contract(off)
  const double s = a.hi + x;
  const double z = s - a.hi;
  const double e = (a.hi - (s - z)) + (x - z);
  a.hi = s;
  a.lo += e;
}
__device__ inline void d2_fma(dd2& a, double x, double y) {
#pragma clang fp contract(off)
  const double p = x * y;
  const double ep = fma(x, y, -p);
  d2_add(a, p);
  a.lo += ep;
}
__device__ inline void d2_merge(dd2& a, const dd2& b) {
#pragma clang fp contract(off)
  d2_add(a, b.hi);
  a.lo += b.lo;
}
__device__ inline double d2_round(const dd2& a) {
#pragma clang fp contract(off)
  return a.hi + a.lo;
}

template <bool CPLX> struct Dd {
  dd2 c[CPLX ? 2 : 1];
};

// acc += conj(a) u (CONJ) or a u, a promoted to FP64
template <bool CONJ, typename V, typename W>
__device__ inline void d2_mac(Dd<VT<W>::cplx>& acc, const V& a, const W& u) {
  if constexpr (VT<W>::cplx) {
    const double ar = (double)vre(a), ai = (double)vim(a), ur = vre(u), ui = vim(u);
    d2_fma(acc.c[0], ar, ur);
    d2_fma(acc.c[0], CONJ ? ai : -ai, ui);
    d2_fma(acc.c[1], ar, ui);
    d2_fma(acc.c[1], CONJ ? -ai : ai, ur);
  } else {
    d2_fma(acc.c[0], (double)vre(a), (double)vre(u));
  }
}

// one-touch load of a streamed entry (non-temporal)
template <typename V> __device__ __forceinline__ V ld_nt(const V* p) {
  if constexpr (VT<V>::cplx) {
    using R = typename VT<V>::real;
    const R* q = reinterpret_cast<const R*>(p);
    return V{__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1)};
  } else {
    return __builtin_nontemporal_load(p);
  }
}

// sum over the wave (butterfly), then lane 0's value for every lane
__device__ inline dd2 d2_wave_sum(dd2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) d2_merge(v, dd2{__shfl_xor(v.hi, off, 64), __shfl_xor(v.lo, off, 64)});
  return dd2{__shfl(v.hi, 0, 64), __shfl(v.lo, 0, 64)};
}

}  // namespace

template <typename V, typename W, int RPT, int WPC, int TPB>
__global__ void __launch_bounds__(TPB) k_resid_tall(const V* __restrict__ At, int64_t ldt, int64_t m, int64_t n,
                                                    const W* __restrict__ y, W* __restrict__ x_out,
                                                    W* __restrict__ qh, W* __restrict__ ql) {
  constexpr bool CP = VT<W>::cplx;
  constexpr int NC = CP ? 2 : 1;
  constexpr int NW = TPB / 64, NG = NW / WPC, SLAB = 64 * RPT;
  __shared__ dd2 red[2][NG][WPC][NC];
  __shared__ dd2 qs[WPC * SLAB][NC];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int gc = wv / WPC, w = wv % WPC;
  const int64_t r0 = (int64_t)w * SLAB;
  const int kmax = (int)(ldt - r0 > 0 ? ((ldt - r0) / 64 < RPT ? (ldt - r0) / 64 : RPT) : 0);
  W yr[RPT];
  Dd<CP> q[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int64_t r = r0 + 64 * k + lane;
    yr[k] = r < m ? y[r] : vzero<W>();
    q[k] = Dd<CP>{};
  }
  const int64_t groups = (int64_t)gridDim.x * NG;
  const int64_t gid = (int64_t)blockIdx.x * NG + gc;
  const int64_t steps = ceil_div(n, groups);
  auto load = [&](V (&x)[RPT], int64_t s) {
    const int64_t c = s * groups + gid;
    const V* col = At + c * ldt + r0 + lane;
#pragma unroll
    for (int k = 0; k < RPT; ++k)
      x[k] = (c < n && k < kmax && r0 + 64 * k + lane < m) ? ld_nt(col + 64 * k) : vzero<V>();
  };
  int slot = 0;
  auto process = [&](const V (&x)[RPT], int64_t s) {
    const int64_t c = s * groups + gid;
    Dd<CP> a{};
#pragma unroll
    for (int k = 0; k < RPT; ++k) d2_mac<true>(a, x[k], yr[k]);
#pragma unroll
    for (int i = 0; i < NC; ++i) a.c[i] = d2_wave_sum(a.c[i]);
    if constexpr (WPC > 1) {
      if (lane == 0)
#pragma unroll
        for (int i = 0; i < NC; ++i) red[slot][gc][w][i] = a.c[i];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        dd2 v = red[slot][gc][0][i];
#pragma unroll
        for (int ww = 1; ww < WPC; ++ww) d2_merge(v, red[slot][gc][ww][i]);
        a.c[i] = v;
      }
      slot ^= 1;
    }
    W wc;
    if constexpr (CP) wc = W{d2_round(a.c[0]), d2_round(a.c[1])};
    else wc = d2_round(a.c[0]);
    if (x_out != nullptr && w == 0 && lane == 0 && c < n) x_out[c] = wc;
#pragma unroll
    for (int k = 0; k < RPT; ++k) d2_mac<false>(q[k], x[k], wc);
  };
  V xa[RPT], xb[RPT];
  if (steps > 0) load(xa, 0);
  for (int64_t s = 0; s < steps; s += 2) {
    if (s + 1 < steps) load(xb, s + 1);
    process(xa, s);
    if (s + 1 < steps) {
      if (s + 2 < steps) load(xa, s + 2);
      process(xb, s + 1);
    }
  }
  // the groups' q, merged in group order, then this workgroup's (hi, lo)
  for (int g2 = 0; g2 < NG; ++g2) {
    __syncthreads();
    if (gc == g2)
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = w * SLAB + 64 * k + lane;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (g2 == 0) qs[i][c] = q[k].c[c];
          else d2_merge(qs[i][c], q[k].c[c]);
        }
      }
  }
  __syncthreads();
  for (int64_t r = t; r < m; r += TPB) {
    const int64_t o = (int64_t)blockIdx.x * m + r;
    if constexpr (CP) {
      qh[o] = W{qs[r][0].hi, qs[r][1].hi};
      ql[o] = W{qs[r][0].lo, qs[r][1].lo};
    } else {
      qh[o] = qs[r][0].hi;
      ql[o] = qs[r][0].lo;
    }
  }
}

// q[i] = the workgroups' (hi, lo) partials merged in a fixed order, rounded
// once: 16 rows per workgroup, the 16 lane groups of a row each merge every
// sixteenth partial, then the group sums are merged in group order.
// grid ceil(m / 16), 256 threads.
template <typename W>
__global__ void __launch_bounds__(256) k_resid_fold(const W* __restrict__ qh, const W* __restrict__ ql, int G,
                                                    int64_t m, W* __restrict__ q) {
  __shared__ dd2 red[2][16][16];
  const int rr = threadIdx.x & 15, part = threadIdx.x >> 4;
  const int64_t i = (int64_t)blockIdx.x * 16 + rr;
  dd2 re{0.0, 0.0}, im{0.0, 0.0};
  if (i < m)
    for (int g = part; g < G; g += 16) {
      const W h = qh[(int64_t)g * m + i], l = ql[(int64_t)g * m + i];
      d2_merge(re, dd2{vre(h), vre(l)});
      if constexpr (VT<W>::cplx) d2_merge(im, dd2{vim(h), vim(l)});
    }
  red[0][part][rr] = re;
  red[1][part][rr] = im;
  __syncthreads();
  if (part == 0 && i < m) {
    for (int k = 1; k < 16; ++k) {
      d2_merge(re, red[0][k][rr]);
      d2_merge(im, red[1][k][rr]);
    }
    q[i] = vmake<W>(d2_round(re), d2_round(im));
  }
}

template <typename V, typename W>
static hipError_t resid_t(const void* At, int64_t ldt, int64_t m, int64_t n, const void* y, void* x_out, void* part,
                          int G, void* q, hipStream_t st) {
  const V* a = reinterpret_cast<const V*>(At);
  const W* yy = reinterpret_cast<const W*>(y);
  W* xo = reinterpret_cast<W*>(x_out);
  W* qh = reinterpret_cast<W*>(part);
  W* ql = qh + (int64_t)G * m;
  if (m <= 512)
    hipLaunchKernelGGL((k_resid_tall<V, W, 8, 1, 256>), dim3((unsigned)G), dim3(256), 0, st, a, ldt, m, n, yy, xo, qh,
                       ql);
  else if (m <= 1024)
    hipLaunchKernelGGL((k_resid_tall<V, W, 8, 2, 256>), dim3((unsigned)G), dim3(256), 0, st, a, ldt, m, n, yy, xo, qh,
                       ql);
  else
    hipLaunchKernelGGL((k_resid_tall<V, W, 8, 4, 256>), dim3((unsigned)G), dim3(256), 0, st, a, ldt, m, n, yy, xo, qh,
                       ql);
  hipLaunchKernelGGL((k_resid_fold<W>), dim3((unsigned)ceil_div(m, 16)), dim3(256), 0, st, qh, ql, G, m,
                     reinterpret_cast<W*>(q));
  return hipGetLastError();
}

int64_t resid_part_elems(int64_t m, int G) { return 2 * (int64_t)G * m; }

hipError_t launch_resid_tall(int dtype, const void* At, int64_t ldt, int64_t m, int64_t n, const void* y, void* x_out,
                             void* part, int G, void* q, hipStream_t st) {
  if (m > kGramTallMaxRows || ldt < m || ldt % 64 != 0 || G < 1) return hipErrorInvalidValue;
  switch (dtype) {
    case 0: return resid_t<cd, cd>(At, ldt, m, n, y, x_out, part, G, q, st);
    case 1: return resid_t<cf, cd>(At, ldt, m, n, y, x_out, part, G, q, st);
    case 2: return resid_t<double, double>(At, ldt, m, n, y, x_out, part, G, q, st);
    case 3: return resid_t<float, double>(At, ldt, m, n, y, x_out, part, G, q, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace mn
