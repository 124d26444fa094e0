// Step 2's factorisation of the l x m sketch, S = Q_S R, by Householder
// reflections (Section 4, Step 2), keeping only R -- the preconditioner of
// Step 4.  Q_S is never formed.
//
// Tiled ("communication-avoiding") Householder QR on 32 x 32 tiles.  For
// each tile column k:
//   level 0   every tile (i, k), i >= k, is reduced to a triangle R_i by its
//             own reflectors; the same reflectors update tiles (i, j), j > k;
//   level s   the triangles are merged pairwise in a binary tree: [R_a; R_b]
//             is reduced to one triangle by reflectors that touch only the
//             pivot row of R_a and the upper triangle of R_b, and the same
//             reflectors update the row-tile pair (a, j), (b, j), j > k.
// Every workgroup (pair, j) recomputes the small factorisation it needs, so
// one launch covers a whole level and no reflector is ever stored globally.
// The triangles live in a ping-pong buffer; the final one of column k is R's
// diagonal block k, and tile (k, j), j > k, ends as R's block (k, j).
//
// Reflector convention: H = I - tau v v^*, v[pivot] = 1, chosen so that
// H^* x = beta e_pivot with beta real and of sign opposite to Re(x_pivot).
// R is unique up to a diagonal unitary factor; its diagonal comes out real.
//
// Ragged sizes: the sketch is copied into an lp x mp tile-aligned matrix
// [[S, 0], [0, 0], [0, I]] whose R is diag(R_S, +-I), so the leading m x m
// block is exactly R_S.
#include "common.hpp"
#include "kernels.hpp"
#include "batch_dev.hpp"

namespace mn {

constexpr int NB = kQrTile;  // 32
constexpr int LDT = NB + 1;  // LDS column stride of a tile (breaks bank conflicts)

// 1/x: hardware reciprocal estimate plus two Newton-Raphson steps
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ inline float recip(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  r = fmaf(r, fmaf(-x, r, 1.0f), r);
  return r;
}

// Householder vector for x = [alpha; rest], |rest|^2 = xn2: returns beta,
// tau and scal = 1 / (alpha - beta) (v_rest = rest * scal).
template <typename V>
__device__ inline void make_reflector(V alpha, typename VT<V>::real xn2, V& tau, typename VT<V>::real& beta,
                                      V& scal) {
  using R = typename VT<V>::real;
  const R ar = vre(alpha), ai = vim(alpha);
  if (xn2 == (R)0 && ai == (R)0) {
    tau = vzero<V>();
    beta = ar;
    scal = vzero<V>();
    return;
  }
  const R nrm = sqrt(ar * ar + ai * ai + xn2);
  beta = ar >= (R)0 ? -nrm : nrm;
  // tau = (beta - alpha) / beta, scal = 1 / (alpha - beta); the reciprocals
  // are hardware estimates refined by two Newton steps (the arguments are
  // positive and far from the range limits: beta is a norm, den >= beta^2)
  const R ib = recip(beta);
  tau = vmake<V>((beta - ar) * ib, -ai * ib);
  const R dr = ar - beta, di = ai;
  const R iden = recip(dr * dr + di * di);
  scal = vmake<V>(dr * iden, -di * iden);
}

// ---------------------------------------------------------------------------
// Tile factorisations in LDS (column stride LDT) by all four waves.  Wave w
// owns columns 8w .. 8w+7; lane (g = lane % 8, cl = lane / 8) owns column
// 8w + cl and rows 4g .. 4g+3, so the sums over a column's rows are DPP
// reductions over 8 adjacent lanes.  Each wave recomputes the pivot column's
// reflector from LDS (bitwise identical in every lane), so one barrier per
// column step suffices.

// Reduce the NB x NB tile T (LDS) to upper-triangular form: on exit beta on
// the diagonal, v below it, tau[] the scalars.  All 256 threads; the tile
// must be in LDS and visible (barrier) before the call.
template <typename V>
__device__ void geqrt_lds(V* T, V* tau) {
  using R = typename VT<V>::real;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane & 7, c = 8 * w + (lane >> 3);
  for (int j = 0; j < NB; ++j) {
    // all of this step's LDS reads first: pivot column, alpha, own column
    V pk[4], o[4];
    const bool upd = c > j;
#pragma unroll
    for (int k = 0; k < 4; ++k) pk[k] = T[(4 * g + k) + j * LDT];
    const V alpha = T[j + j * LDT];
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = upd ? T[(4 * g + k) + c * LDT] : vzero<V>();
    R part = (R)0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (4 * g + k > j) part += vabs2(pk[k]);
    const R xn2 = sum8(part);
    V tj, sc;
    R bt;
    make_reflector<V>(alpha, xn2, tj, bt, sc);
    V vk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = 4 * g + k;
      vk[k] = (r == j) ? vmake<V>(1.0, 0.0) : (r > j ? vmul(pk[k], sc) : vzero<V>());
    }
    V wsum = vzero<V>();
#pragma unroll
    for (int k = 0; k < 4; ++k) wsum = vcfma(vk[k], o[k], wsum);
    wsum = sum8(wsum);
    const V f = vmul(vconj(tj), wsum);
    if (upd) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (4 * g + k >= j) T[(4 * g + k) + c * LDT] = vsub(o[k], vmul(vk[k], f));
    }
    // every wave has read column j: its owner may now overwrite it; column
    // j+1, read next, was finished above by its owner
    __syncthreads();
    if (c == j) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = 4 * g + k;
        if (r > j) T[r + j * LDT] = vk[k];
        else if (r == j) T[j + j * LDT] = vmake<V>((double)bt, 0.0);
      }
    }
    if (threadIdx.x == 0) tau[j] = tj;
  }
  __syncthreads();
}

// Merge two triangles in LDS: [R1; R2] -> R1 new triangle, R2's upper part
// the reflector tails v2, tau[] the scalars.  All 256 threads; inputs must be
// in LDS and visible before the call.
template <typename V>
__device__ void ttqrt_lds(V* R1, V* R2, V* tau) {
  using R = typename VT<V>::real;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane & 7, c = 8 * w + (lane >> 3);
  for (int j = 0; j < NB; ++j) {
    // all of this step's LDS reads first: pivot column, alpha, own column
    V pk[4], o[4];
    const bool upd = c > j;
#pragma unroll
    for (int k = 0; k < 4; ++k) pk[k] = (4 * g + k <= j) ? R2[(4 * g + k) + j * LDT] : vzero<V>();
    const V alpha = R1[j + j * LDT];
    const V top = (upd && g == 0) ? R1[j + c * LDT] : vzero<V>();
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = upd ? R2[(4 * g + k) + c * LDT] : vzero<V>();
    R part = (R)0;
#pragma unroll
    for (int k = 0; k < 4; ++k) part += vabs2(pk[k]);
    const R xn2 = sum8(part);
    V tj, sc;
    R bt;
    make_reflector<V>(alpha, xn2, tj, bt, sc);
    V vk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) vk[k] = vmul(pk[k], sc);
    V wsum = top;
#pragma unroll
    for (int k = 0; k < 4; ++k) wsum = vcfma(vk[k], o[k], wsum);
    wsum = sum8(wsum);
    const V f = vmul(vconj(tj), wsum);
    if (upd) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (4 * g + k <= j) R2[(4 * g + k) + c * LDT] = vsub(o[k], vmul(vk[k], f));
      if (g == 0) R1[j + c * LDT] = vsub(top, f);
    }
    // every wave has read column j: its owner may now overwrite it
    __syncthreads();
    if (c == j) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (4 * g + k <= j) R2[(4 * g + k) + j * LDT] = vk[k];
      if (g == 0) R1[j + j * LDT] = vmake<V>((double)bt, 0.0);
    }
    if (threadIdx.x == 0) tau[j] = tj;
  }
  __syncthreads();
}

// Apply Q^* of a geqrt'd tile (reflectors in T, tau) to the tile C held in
// registers: thread t owns column t/8, rows 4*(t%8) .. +3.
template <typename V>
__device__ inline void apply_geqrt(const V* T, const V* tau, V* c) {
  const int t = threadIdx.x;
  const int q0 = (t & 7) * 4;
  for (int r = 0; r < NB; ++r) {
    V part = vzero<V>();
    V vq[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = q0 + u;
      vq[u] = (q == r) ? vmake<V>(1.0, 0.0) : (q > r ? T[q + r * LDT] : vzero<V>());
      part = vcfma(vq[u], c[u], part);
    }
    part = sum8(part);
    const V f = vmul(vconj(tau[r]), part);
#pragma unroll
    for (int u = 0; u < 4; ++u) c[u] = vsub(c[u], vmul(vq[u], f));
  }
}

// Apply the merge's Q^* to the row-tile pair (C1 top, C2 bottom) held in
// registers: thread t owns column t/8, rows 4*(t%8)..+3 of both tiles.
template <typename V>
__device__ inline void apply_ttqrt(const V* V2, const V* tau, V* c1, V* c2) {
  const int t = threadIdx.x;
  const int q0 = (t & 7) * 4;
  for (int r = 0; r < NB; ++r) {
    V part = vzero<V>();
    const bool own_top = (r >> 2) == (t & 7);
    V vq[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = q0 + u;
      vq[u] = (q <= r) ? V2[q + r * LDT] : vzero<V>();
      part = vcfma(vq[u], c2[u], part);
      if (own_top && q == r) part = vadd(part, c1[u]);
    }
    part = sum8(part);
    const V f = vmul(vconj(tau[r]), part);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = q0 + u;
      if (own_top && q == r) c1[u] = vsub(c1[u], f);
      c2[u] = vsub(c2[u], vmul(vq[u], f));
    }
  }
}

// tile load / store (column-major, leading dimension ld), all 256 threads
template <typename V> __device__ inline void tile_to_lds(V* dst, const V* src, int64_t ld) {
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) dst[(e % NB) + (e / NB) * LDT] = src[(e % NB) + (int64_t)(e / NB) * ld];
}
template <typename V> __device__ inline void tile_from_lds(V* dst, int64_t ld, const V* src) {
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) dst[(e % NB) + (int64_t)(e / NB) * ld] = src[e];
}
// LDS tile (stride LDT) -> contiguous NB x NB upper triangle in global memory
template <typename V> __device__ inline void triu_store(V* dst, const V* src) {
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    const int r = e % NB, c = e / NB;
    dst[e] = r <= c ? src[r + c * LDT] : vzero<V>();
  }
}
template <typename V> __device__ inline void regs_load(V* c, const V* tile, int64_t ld) {
  const int col = threadIdx.x >> 3, q0 = (threadIdx.x & 7) * 4;
#pragma unroll
  for (int u = 0; u < 4; ++u) c[u] = tile[(q0 + u) + (int64_t)col * ld];
}
template <typename V> __device__ inline void regs_store(V* tile, int64_t ld, const V* c) {
  const int col = threadIdx.x >> 3, q0 = (threadIdx.x & 7) * 4;
#pragma unroll
  for (int u = 0; u < 4; ++u) tile[(q0 + u) + (int64_t)col * ld] = c[u];
}

// ---------------------------------------------------------------------------
// copy S (l x m, lds) into the tile-aligned Sp (lp x mp, ld lp)
template <typename V>
__global__ void k_qr_pad(const V* __restrict__ S, int64_t lds, int64_t l, int64_t m, V* __restrict__ Sp, int64_t lp,
                         int64_t mp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= lp * mp) return;
  const int64_t r = e % lp, c = e / lp;
  V v = vzero<V>();
  if (r < l && c < m) v = S[r + c * lds];
  else if (c >= m && r == lp - (mp - m) + (c - m)) v = vmake<V>(1.0, 0.0);
  Sp[e] = v;
}

// level 0 of tile column k: grid (MT - k, NT - k), 256 threads
template <typename V>
__global__ void __launch_bounds__(256) k_qr_level0(V* __restrict__ Sp, int64_t lp, int k, V* __restrict__ Rb,
                                                   V* __restrict__ Rdiag, int write_diag) {
  __shared__ V T[LDT * NB];
  __shared__ V tau[NB];
  const int i = k + blockIdx.x;
  const int jj = blockIdx.y;
  const V* tile_ik = Sp + (int64_t)i * NB + (int64_t)k * NB * lp;
  V* tile_ij = Sp + (int64_t)i * NB + (int64_t)(k + jj) * NB * lp;
  V c[4];
  if (jj != 0) regs_load(c, tile_ij, lp);  // in flight during the factorisation
  tile_to_lds(T, tile_ik, lp);
  __syncthreads();
  geqrt_lds<V>(T, tau);
  if (jj == 0) {
    triu_store(Rb + (int64_t)i * NB * NB, T);
    if (write_diag) triu_store(Rdiag + (int64_t)k * NB * NB, T);
    return;
  }
  apply_geqrt<V>(T, tau, c);
  regs_store(tile_ij, lp, c);
}

// tree level s of tile column k: grid (pairs, NT - k), 256 threads
template <typename V>
__global__ void __launch_bounds__(256) k_qr_tree(V* __restrict__ Sp, int64_t lp, int MT, int k, int s,
                                                 const V* __restrict__ Rin, V* __restrict__ Rout,
                                                 V* __restrict__ Rdiag, int final_level) {
  __shared__ V R1[LDT * NB];
  __shared__ V R2[LDT * NB];
  __shared__ V tau[NB];
  const int p = blockIdx.x;
  const int jj = blockIdx.y;
  const int i1 = k + p * (2 << s);
  const int i2 = i1 + (1 << s);
  if (i2 >= MT) {
    if (jj == 0)
      for (int e = threadIdx.x; e < NB * NB; e += blockDim.x)
        Rout[(int64_t)i1 * NB * NB + e] = Rin[(int64_t)i1 * NB * NB + e];
    return;
  }
  V* t1 = Sp + (int64_t)i1 * NB + (int64_t)(k + jj) * NB * lp;
  V* t2 = Sp + (int64_t)i2 * NB + (int64_t)(k + jj) * NB * lp;
  V c1[4], c2[4];
  if (jj != 0) {  // in flight during the factorisation
    regs_load(c1, t1, lp);
    regs_load(c2, t2, lp);
  }
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    R1[(e % NB) + (e / NB) * LDT] = Rin[(int64_t)i1 * NB * NB + e];
    R2[(e % NB) + (e / NB) * LDT] = Rin[(int64_t)i2 * NB * NB + e];
  }
  __syncthreads();
  ttqrt_lds<V>(R1, R2, tau);
  if (jj == 0) {
    triu_store(Rout + (int64_t)i1 * NB * NB, R1);
    if (final_level) triu_store(Rdiag + (int64_t)k * NB * NB, R1);
    return;
  }
  apply_ttqrt<V>(R2, tau, c1, c2);
  regs_store(t1, lp, c1);
  regs_store(t2, lp, c2);
}

// R (m x m, ldr) from the diagonal triangles and the tiles (I, J), I < J;
// also max and min of |R_ii| (i < m) into dmax[0], dmax[1] via a second kernel.
template <typename V>
__global__ void k_qr_extract(const V* __restrict__ Sp, int64_t lp, const V* __restrict__ Rdiag, int64_t m,
                             V* __restrict__ Rout, int64_t ldr) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * m) return;
  const int64_t r = e % m, c = e / m;
  V v = vzero<V>();
  if (r <= c) {
    const int64_t I = r / NB, J = c / NB;
    if (I == J) v = Rdiag[I * NB * NB + (r % NB) + (c % NB) * NB];
    else v = Sp[r + c * lp];
  }
  Rout[r + c * ldr] = v;
}

template <typename V>
__device__ __forceinline__ void k_rdiag_range_body(const Bk bk, const V* __restrict__ R, int64_t ldr, int64_t m, double* __restrict__ out) {
  __shared__ double red[16];
  double mx = 0.0, mn = 1.0e308;
  bool fin = true;
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
    const V d = R[i + i * ldr];
    const double a = sqrt((double)vabs2(d));
    fin = fin && vfinite(d);
    mx = fmax(mx, a);
    mn = fmin(mn, a);
  }
  mx = block_max(mx, red);
  mn = -block_max(-mn, red);
  double f = fin ? 0.0 : 1.0;
  f = block_max(f, red);
  if (threadIdx.x == 0) {
    out[0] = mx;
    out[1] = mn;
    out[2] = f;
  }
}
template <typename V>
__global__ void k_rdiag_range(const V* __restrict__ R, int64_t ldr, int64_t m, double* __restrict__ out) {
  k_rdiag_range_body<V>(bk_hw(), R, ldr, m, out);
}

template <typename V>
static hipError_t qr_impl(const QrArgs& a, hipStream_t st) {
  const int64_t mp = ceil_div(a.m, NB) * NB;
  const int64_t lp = ceil_div(a.l + (mp - a.m), NB) * NB;
  const int MT = (int)(lp / NB), NT = (int)(mp / NB);
  V* Sp = reinterpret_cast<V*>(a.work);
  V* Rb0 = Sp + lp * mp;
  V* Rb1 = Rb0 + (int64_t)MT * NB * NB;
  V* Rdiag = Rb1 + (int64_t)MT * NB * NB;
  hipLaunchKernelGGL((k_qr_pad<V>), dim3((unsigned)ceil_div(lp * mp, 256)), dim3(256), 0, st,
                     reinterpret_cast<const V*>(a.S), a.lds, a.l, a.m, Sp, lp, mp);
  for (int k = 0; k < NT; ++k) {
    const int span = MT - k;
    hipLaunchKernelGGL((k_qr_level0<V>), dim3(span, NT - k), dim3(256), 0, st, Sp, lp, k, Rb0, Rdiag,
                       span == 1 ? 1 : 0);
    V* rin = Rb0;
    V* rout = Rb1;
    for (int s = 0; (1 << s) < span; ++s) {
      const int pairs = (int)ceil_div(span, 2 << s);
      const int fin = (2 << s) >= span ? 1 : 0;
      hipLaunchKernelGGL((k_qr_tree<V>), dim3(pairs, NT - k), dim3(256), 0, st, Sp, lp, MT, k, s, rin, rout, Rdiag,
                         fin);
      V* tmp = rin;
      rin = rout;
      rout = tmp;
    }
  }
  V* R = reinterpret_cast<V*>(a.R);
  hipLaunchKernelGGL((k_qr_extract<V>), dim3((unsigned)ceil_div(a.m * a.m, 256)), dim3(256), 0, st, Sp, lp, Rdiag,
                     a.m, R, a.ldr);
  hipLaunchKernelGGL((k_rdiag_range<V>), dim3(1), dim3(1024), 0, st, R, a.ldr, a.m, a.diag_out);
  return hipGetLastError();
}

int64_t qr_work_bytes(int dtype, int64_t l, int64_t m) {
  const int64_t mp = ceil_div(m, NB) * NB;
  const int64_t lp = ceil_div(l + (mp - m), NB) * NB;
  const int64_t MT = lp / NB, NT = mp / NB;
  const int64_t elems = lp * mp + 2 * MT * NB * NB + NT * NB * NB;
  return elems * dtype_size(dtype);
}

hipError_t launch_rdiag_range(int dtype, const void* R, int64_t ldr, int64_t m, double* out, hipStream_t st) {
  switch (dtype) {
    case 0: hipLaunchKernelGGL((k_rdiag_range<cd>), dim3(1), dim3(1024), 0, st, (const cd*)R, ldr, m, out); break;
    case 1: hipLaunchKernelGGL((k_rdiag_range<cf>), dim3(1), dim3(1024), 0, st, (const cf*)R, ldr, m, out); break;
    case 2: hipLaunchKernelGGL((k_rdiag_range<double>), dim3(1), dim3(1024), 0, st, (const double*)R, ldr, m, out); break;
    case 3: hipLaunchKernelGGL((k_rdiag_range<float>), dim3(1), dim3(1024), 0, st, (const float*)R, ldr, m, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_qr(int dtype, const QrArgs& a, hipStream_t st) {
  switch (dtype) {
    case 0: return qr_impl<cd>(a, st);
    case 1: return qr_impl<cf>(a, st);
    case 2: return qr_impl<double>(a, st);
    case 3: return qr_impl<float>(a, st);
  }
  return hipErrorInvalidValue;
}

namespace {
template <typename V>
__global__ void kb_rdiag(const BSys* __restrict__ sys, const BGrid* __restrict__ grid, int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_rdiag_range_body<V>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<const V*>(s.R), s.m,
                        s.m, s.diag);
}
}  // namespace

hipError_t launch_b_rdiag(bool cplx, const BLaunch& L, hipStream_t st) {
  if (cplx) hipLaunchKernelGGL(kb_rdiag<cd>, dim3((unsigned)L.total), dim3(1024), 0, st, L.sys, L.grid, L.nsys);
  else hipLaunchKernelGGL(kb_rdiag<double>, dim3((unsigned)L.total), dim3(1024), 0, st, L.sys, L.grid, L.nsys);
  return hipGetLastError();
}

}  // namespace mn
