// R with R* R = G for the Hermitian positive definite Gram matrix G = S* S of
// the sketch (Section 4, Step 2 uses only the triangular factor of S: R* R =
// S* S holds for the R of any QR decomposition S = Q R).
//
// Right-looking blocked Cholesky on 32 x 32 tiles, one launch per block step
// k.  The diagonal tile is factored once, by the workgroup that applies its
// last update in step k - 1, which also stores R_kk^{-*}; step k then forms
//   tile (k, j), j > k:         R_kj = R_kk^{-*} G_kj      (written to R)
//   tile (i, j), k < i <= j:    G_ij -= R_ki^* R_kj        (Schur complement)
// as plain 32 x 32 products, recomputing the R_k* tiles it needs.  G tiles of
// block row k are only read during step k, so R goes to a separate buffer and
// no step races with itself.  FP64 throughout.
#include "common.hpp"
#include "kernels.hpp"
#include "batch_dev.hpp"

namespace mn {

namespace {

constexpr int CB = 32;        // tile edge
constexpr int LDC = CB + 1;   // LDS column stride

// tile (row block bi, column block bj) of a column-major matrix -> LDS, zero
// outside the m x m matrix
template <typename V>
__device__ void tile_in(V* T, const V* G, int64_t ld, int64_t m, int bi, int bj) {
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
    const int r = e % CB, c = e / CB;
    const int64_t gr = (int64_t)bi * CB + r, gc = (int64_t)bj * CB + c;
    T[r + c * LDC] = (gr < m && gc < m) ? G[gr + gc * ld] : vzero<V>();
  }
}

// In place: T (upper part of a Hermitian tile) -> its Cholesky factor R (upper),
// T = R* R, and Z (LDS, 32 x 32) -> R^{-*}.  Padding rows/columns beyond
// `valid` are set to the identity so the factor stays invertible.  Step c
// subtracts conj(T_ci)/T_cc times row c from every row i > c (right-looking
// elimination T = L D L*, upper part only), and the same row operations turn
// Z = I into L^{-1}; at the end the rows of T are scaled to R = D^{1/2} L*
// and those of Z to R^{-*} = D^{-1/2} L^{-1}.  (Column q of L^{-1} receives
// exactly the operations of a forward substitution L z = e_q.)
// Thread t keeps its elements (i, j) = (t % 32, t / 32 + 8u) of T and Z in
// registers; at step c the threads of row c publish that row to a small
// double-buffered LDS row (one barrier per step), which every thread reads.
// rinv[i] = 1 / R_ii.  Returns false if a pivot is not positive and finite.
template <typename V>
__device__ __forceinline__ bool chol_tile(V* T, V* Z, int valid, double* piv, double* rinv) {
  __shared__ V rowT[2][CB];
  __shared__ V rowZ[2][CB];
  const int i = threadIdx.x % CB, jb = threadIdx.x / CB;  // rows i, columns jb + 8u
  V t[4], z[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = jb + 8 * u;
    t[u] = (i >= valid || j >= valid) ? ((i == j) ? vmake<V>(1.0, 0.0) : vzero<V>()) : T[i + j * LDC];
    z[u] = (i == j) ? vmake<V>(1.0, 0.0) : vzero<V>();
  }
  for (int c = 0; c < CB; ++c) {
    const int buf = c & 1;
    if (i == c) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        rowT[buf][jb + 8 * u] = t[u];
        rowZ[buf][jb + 8 * u] = z[u];
      }
    }
    __syncthreads();
    const double d = vre(rowT[buf][c]);
    const V tci = rowT[buf][i];
    V tcj[4], zcq[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      tcj[u] = rowT[buf][jb + 8 * u];
      zcq[u] = rowZ[buf][jb + 8 * u];
    }
    if (threadIdx.x == 0) piv[c] = d;
    const double inv = 1.0 / d;
    const V f = vscale(vconj(tci), inv);  // multiplier of row c for row i
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = jb + 8 * u;
      if (i > c && i <= j) t[u] = vsub(t[u], vmul(f, tcj[u]));
      if (i > c && j <= c) z[u] = vsub(z[u], vmul(f, zcq[u]));
    }
  }
  __syncthreads();
  bool ok = true;
  for (int c = 0; c < CB; ++c) ok = ok && (piv[c] > 0.0) && isfinite(piv[c]);
  const double pi = piv[i];
  const double s = pi > 0.0 ? 1.0 / sqrt(pi) : 0.0;
  if (jb == 0) rinv[i] = s;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = jb + 8 * u;
    if (i < j) T[i + j * LDC] = vscale(t[u], s);
    else if (i == j) T[i + j * LDC] = vmake<V>(pi > 0.0 ? sqrt(pi) : 0.0, 0.0);
    else T[i + j * LDC] = vzero<V>();
    Z[i + j * LDC] = vscale(z[u], s);
  }
  __syncthreads();
  return ok;
}

// acc[u] = sum_q A(r, q) B(q, cg + 8u) for tiles in LDS; thread t takes row
// r = t % 32 and columns cg + 8u, cg = t / 32.
template <typename V>
__device__ __forceinline__ void tile_mm(const V* A, const V* B, V acc[4]) {
  const int r = threadIdx.x % CB, cg = threadIdx.x / CB;
#pragma unroll 8
  for (int q = 0; q < CB; ++q) {
    const V a = A[r + q * LDC];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = vfma(a, B[q + (cg + 8 * u) * LDC], acc[u]);
  }
}

// Factor the (updated) diagonal tile held in T for block k: R_kk -> R,
// Y_kk = R_kk^{-*} -> Yd[k] (32 x 32, column-major, ld 32); Y is LDS scratch.
// The strictly lower blocks of R are zeroed by the panel workgroups.
// With X, also X_kk = R_kk^{-1} = Y_kk^* (the whole 32 x 32 block, identity
// beyond m, so X is padded to whole blocks).
template <typename V>
__device__ __forceinline__ void finish_diag(V* T, V* Y, double* piv, double* rinv, int k, int64_t m, V* R,
                                            int64_t ldr, V* Yd, V* X, int64_t ldx, int32_t* bad) {
  const int valid = (int)((m - (int64_t)k * CB) < CB ? (m - (int64_t)k * CB) : CB);
  const bool ok = chol_tile(T, Y, valid, piv, rinv);
  if (!ok && threadIdx.x == 0) bad[0] = 1;
  const int r = threadIdx.x % CB, cg = threadIdx.x / CB;
  V* yd = Yd + (int64_t)k * CB * CB;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = cg + 8 * u;
    const int64_t gr = (int64_t)k * CB + r, gc = (int64_t)k * CB + c;
    if (gr < m && gc < m) R[gr + gc * ldr] = T[r + c * LDC];
    yd[r + c * CB] = Y[r + c * LDC];
    if (X) X[gr + gc * ldx] = vconj(Y[c + r * LDC]);
  }
}

// Block step s of X = R^{-1}, right-looking (block column s of X final: X_is
// for i <= s): tile (i, j), i <= s < j, adds X_is R_sj to the running sum
// held in X_ij (stored, not added, for its first term s = i); the tiles of
// column j = s + 1 then hold the whole sum S and become X_ij = -S X_jj.
template <typename V>
__device__ __forceinline__ void trtri_tile(int w, int s, int nbk, int64_t m, const V* __restrict__ R, int64_t ldr,
                                           V* __restrict__ X, int64_t ldx, V* As, V* Bs) {
  const int ncol = nbk - s - 1;
  const int i = w / ncol, j = s + 1 + w % ncol;
  const int r = threadIdx.x % CB, cg = threadIdx.x / CB;
  const int64_t mx = (int64_t)nbk * CB;  // X is stored on whole blocks
  V acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
    acc[u] = (s == i) ? vzero<V>() : X[((int64_t)i * CB + r) + ((int64_t)j * CB + cg + 8 * u) * ldx];
  tile_in(As, X, ldx, mx, i, s);  // X_is
  tile_in(Bs, R, ldr, m, s, j);   // R_sj (off the diagonal: zero beyond m)
  __syncthreads();
  tile_mm(As, Bs, acc);
  if (j == s + 1) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) As[r + (cg + 8 * u) * LDC] = acc[u];
    tile_in(Bs, X, ldx, mx, j, j);  // X_jj
    __syncthreads();
    V o[4] = {vzero<V>(), vzero<V>(), vzero<V>(), vzero<V>()};
    tile_mm(As, Bs, o);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = vsub(vzero<V>(), o[u]);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) X[((int64_t)i * CB + r) + ((int64_t)j * CB + cg + 8 * u) * ldx] = acc[u];
}

// Block step 0's diagonal tile (one workgroup).
template <typename V>
__device__ __forceinline__ void k_chol_diag0_body(const Bk bk, V* __restrict__ G, int64_t ldg, int64_t m,
                                                   V* __restrict__ R, int64_t ldr, V* __restrict__ Yd, V* X,
                                                   int64_t ldx, int32_t* __restrict__ bad) {
  (void)bk;
  __shared__ V T[CB * LDC];
  __shared__ V Y[CB * LDC];
  __shared__ double piv[CB];
  __shared__ double rinv[CB];
  tile_in(T, G, ldg, m, 0, 0);
  __syncthreads();
  finish_diag(T, Y, piv, rinv, 0, m, R, ldr, Yd, X, ldx, bad);
}
template <typename V>
__global__ void __launch_bounds__(256) k_chol_diag0(V* __restrict__ G, int64_t ldg, int64_t m, V* __restrict__ R,
                                                    int64_t ldr, V* __restrict__ Yd, V* X, int64_t ldx,
                                                    int32_t* __restrict__ bad) {
  k_chol_diag0_body<V>(bk_hw(), G, ldg, m, R, ldr, Yd, X, ldx, bad);
}

// Block step k (R_kk and Y_kk = R_kk^{-*} known):
//   tile (k, j), j > k:      R_kj = Y_kk G_kj                     -> R
//   tile (i, j), k < i <= j: G_ij -= (Y_kk G_ki)^* (Y_kk G_kj); the workgroup
//                            of (k+1, k+1) then factors it (R, Y of block k+1).
// grid = (nbk - k - 1) + (nbk - k - 1)(nbk - k)/2 workgroups, plus, with X,
// k (nbk - k) workgroups for block step k - 1 of X = R^{-1} (its inputs, R's
// block row k - 1 and X_kk, come from the previous launch; k = nbk - 1 runs
// only those).
//
// SEP: block row k of R comes from a separate launch before this one
// (k_chol_panel), so the grid holds only the trailing tiles (and the X
// workgroups) and each trailing tile reads R_ki, R_kj instead of forming them.
template <typename V, bool SEP = false>
__device__ __forceinline__ void k_chol_step_body(const Bk bk, V* __restrict__ G, int64_t ldg, int64_t m, int k, int nbk,
                                                   V* __restrict__ R, int64_t ldr, V* __restrict__ Yd, V* X,
                                                   int64_t ldx, int32_t* __restrict__ bad) {
  __shared__ V Y[CB * LDC];
  __shared__ V TA[CB * LDC];
  __shared__ V TB[CB * LDC];
  __shared__ double piv[CB];
  __shared__ double rinv[CB];
  const int nrow = nbk - k - 1;
  const int npanel = SEP ? 0 : nrow;
  const int nchol = npanel + nrow * (nrow + 1) / 2;
  if (bk.x >= nchol) {
    trtri_tile(bk.x - nchol, k - 1, nbk, m, R, ldr, X, ldx, TA, TB);
    return;
  }
  int bi, bj;
  int w = bk.x;
  if (w < npanel) {
    bi = k;
    bj = k + 1 + w;
  } else {
    w -= npanel;
    bi = k + 1;
    int len = nbk - bi;
    while (w >= len) {
      w -= len;
      ++bi;
      len = nbk - bi;
    }
    bj = bi + w;
  }
  const int r = threadIdx.x % CB, cg = threadIdx.x / CB;
  const V* yd = Yd + (int64_t)k * CB * CB;
  if (!SEP)
    for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) Y[(e % CB) + (e / CB) * LDC] = yd[e];
  if (!SEP && bi == k) {
    tile_in(TA, G, ldg, m, k, bj);
    __syncthreads();
    V acc[4] = {vzero<V>(), vzero<V>(), vzero<V>(), vzero<V>()};
    tile_mm(Y, TA, acc);  // R_kj
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t gr = (int64_t)k * CB + r, gc = (int64_t)bj * CB + cg + 8 * u;
      if (gr < m && gc < m) R[gr + gc * ldr] = acc[u];
      // the mirrored tile (bj, k) of R's strictly lower part
      const int64_t lr = (int64_t)bj * CB + r, lc = (int64_t)k * CB + cg + 8 * u;
      if (lr < m && lc < m) R[lr + lc * ldr] = vzero<V>();
    }
    return;
  }
  // trailing tile: P = R_ki = Y G_ki, Q = R_kj = Y G_kj; G_ij -= P^* Q.
  // This workgroup's own G_ij is loaded first (no other workgroup writes it
  // in this step).
  V gij[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t gr = (int64_t)bi * CB + r, gc = (int64_t)bj * CB + cg + 8 * u;
    gij[u] = (gr < m && gc < m) ? G[gr + gc * ldg] : vzero<V>();
  }
  if constexpr (SEP) {
    // TA <- R_ki^* (rows of P^* contiguous for the product), TB <- R_kj
    for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
      const int rr = e % CB, cc = e / CB;
      const int64_t gr = (int64_t)k * CB + rr, gci = (int64_t)bi * CB + cc, gcj = (int64_t)bj * CB + cc;
      TA[cc + rr * LDC] = (gr < m && gci < m) ? vconj(R[gr + gci * ldr]) : vzero<V>();
      TB[rr + cc * LDC] = (gr < m && gcj < m) ? R[gr + gcj * ldr] : vzero<V>();
    }
  } else {
  tile_in(TA, G, ldg, m, k, bi);
  if (bj != bi) tile_in(TB, G, ldg, m, k, bj);
  __syncthreads();
  // TA <- P^* (so the product reads rows of P^* contiguously), TB <- Q
  {
    V p[4] = {vzero<V>(), vzero<V>(), vzero<V>(), vzero<V>()};
    tile_mm(Y, TA, p);
    if (bj != bi) {
      V q[4] = {vzero<V>(), vzero<V>(), vzero<V>(), vzero<V>()};
      tile_mm(Y, TB, q);
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 4; ++u) TB[r + (cg + 8 * u) * LDC] = q[u];
    } else {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 4; ++u) TB[r + (cg + 8 * u) * LDC] = p[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) TA[(cg + 8 * u) + r * LDC] = vconj(p[u]);
  }
  }
  __syncthreads();
  V acc[4] = {vzero<V>(), vzero<V>(), vzero<V>(), vzero<V>()};
  tile_mm(TA, TB, acc);
  if (bi == k + 1 && bj == k + 1) {
    // the next diagonal tile is final: factor it for block step k + 1
    __syncthreads();  // TB's reads are done before it is overwritten
#pragma unroll
    for (int u = 0; u < 4; ++u) TB[r + (cg + 8 * u) * LDC] = vsub(gij[u], acc[u]);
    __syncthreads();
    finish_diag(TB, TA, piv, rinv, k + 1, m, R, ldr, Yd, X, ldx, bad);
    return;
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = cg + 8 * u;
    const int64_t gr = (int64_t)bi * CB + r, gc = (int64_t)bj * CB + c;
    if (gr < m && gc < m && gr <= gc) G[gr + gc * ldg] = vsub(gij[u], acc[u]);
  }
}
template <typename V>
__global__ void __launch_bounds__(256) k_chol_step(V* __restrict__ G, int64_t ldg, int64_t m, int k, int nbk,
                                                   V* __restrict__ R, int64_t ldr, V* __restrict__ Yd, V* X,
                                                   int64_t ldx, int32_t* __restrict__ bad) {
  k_chol_step_body<V>(bk_hw(), G, ldg, m, k, nbk, R, ldr, Yd, X, ldx, bad);
}

template <typename V>
__global__ void __launch_bounds__(256) k_chol_step_sep(V* __restrict__ G, int64_t ldg, int64_t m, int k, int nbk,
                                                       V* __restrict__ R, int64_t ldr, V* __restrict__ Yd, V* X,
                                                       int64_t ldx, int32_t* __restrict__ bad) {
  k_chol_step_body<V, true>(bk_hw(), G, ldg, m, k, nbk, R, ldr, Yd, X, ldx, bad);
}

// Block row k of R: tile (k, k + 1 + w) = Y_kk G_k,k+1+w (and its mirrored
// strictly lower tile zeroed).  grid = nbk - k - 1.
template <typename V>
__global__ void __launch_bounds__(256) k_chol_panel(const V* __restrict__ G, int64_t ldg, int64_t m, int k,
                                                    V* __restrict__ R, int64_t ldr, const V* __restrict__ Yd) {
  __shared__ V Y[CB * LDC];
  __shared__ V TA[CB * LDC];
  const int bj = k + 1 + (int)blockIdx.x;
  const int r = threadIdx.x % CB, cg = threadIdx.x / CB;
  const V* yd = Yd + (int64_t)k * CB * CB;
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) Y[(e % CB) + (e / CB) * LDC] = yd[e];
  tile_in(TA, G, ldg, m, k, bj);
  __syncthreads();
  V acc[4] = {vzero<V>(), vzero<V>(), vzero<V>(), vzero<V>()};
  tile_mm(Y, TA, acc);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t gr = (int64_t)k * CB + r, gc = (int64_t)bj * CB + cg + 8 * u;
    if (gr < m && gc < m) R[gr + gc * ldr] = acc[u];
    const int64_t lr = (int64_t)bj * CB + r, lc = (int64_t)k * CB + cg + 8 * u;
    if (lr < m && lc < m) R[lr + lc * ldr] = vzero<V>();
  }
}

// Two launches per block step: block row k of R (k_chol_panel), then the
// trailing tiles, which read it (one 32 x 32 product each instead of three),
// the factorisation of diagonal tile k + 1 and block step k - 1 of X.
template <typename V>
hipError_t chol_impl(void* G, int64_t ldg, int64_t m, void* R, int64_t ldr, void* Yd, void* X, int64_t ldx,
                     int32_t* bad, hipStream_t st) {
  const int nbk = (int)ceil_div(m, CB);
  V* Xv = reinterpret_cast<V*>(X);
  V* Gv = reinterpret_cast<V*>(G);
  V* Rv = reinterpret_cast<V*>(R);
  V* Ydv = reinterpret_cast<V*>(Yd);
  hipLaunchKernelGGL((k_chol_diag0<V>), dim3(1), dim3(256), 0, st, Gv, ldg, m, Rv, ldr, Ydv, Xv, ldx, bad);
  for (int k = 0; k < nbk; ++k) {
    const int nrow = nbk - k - 1;
    const int ntrail = (nbk - k - 1) * (nbk - k) / 2;
    const int ntri = (X && k >= 1) ? k * (nbk - k) : 0;
    if (nrow > 0)
      hipLaunchKernelGGL((k_chol_panel<V>), dim3((unsigned)nrow), dim3(256), 0, st, Gv, ldg, m, k, Rv, ldr, Ydv);
    if (ntrail + ntri == 0) continue;
    hipLaunchKernelGGL((k_chol_step_sep<V>), dim3((unsigned)(ntrail + ntri)), dim3(256), 0, st, Gv, ldg, m, k, nbk,
                       Rv, ldr, Ydv, Xv, ldx, bad);
  }
  return hipGetLastError();
}

}  // namespace

int64_t chol_scratch_elems(int64_t m) { return ceil_div(m, CB) * CB * CB; }

hipError_t launch_chol(bool cplx, void* G, int64_t ldg, int64_t m, void* R, int64_t ldr, void* Yd, void* X,
                       int64_t ldx, int32_t* bad, hipStream_t st) {
  if (m < 1 || ldg < m || ldr < m) return hipErrorInvalidValue;
  if (X && ldx < ceil_div(m, CB) * CB) return hipErrorInvalidValue;
  return cplx ? chol_impl<cd>(G, ldg, m, R, ldr, Yd, X, ldx, bad, st)
              : chol_impl<double>(G, ldg, m, R, ldr, Yd, X, ldx, bad, st);
}

namespace {
template <typename V>
__global__ void __launch_bounds__(256) kb_chol_diag0(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                     int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_chol_diag0_body<V>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<V*>(s.G), s.m, s.m,
                       reinterpret_cast<V*>(s.R), s.m, reinterpret_cast<V*>(s.Yd), (V*)nullptr, 0, s.flags + 1);
}
template <typename V>
__global__ void __launch_bounds__(256) kb_chol_step(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                    int nsys, int k) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_chol_step_body<V>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<V*>(s.G), s.m, s.m, k,
                      (int)ceil_div(s.m, CB), reinterpret_cast<V*>(s.R), s.m, reinterpret_cast<V*>(s.Yd),
                      (V*)nullptr, 0, s.flags + 1);
}
}  // namespace

// k < 0: every system's first diagonal tile (one workgroup each); k >= 0: block
// step k of every system with more than k + 1 block columns
hipError_t launch_b_chol_step(bool cplx, const BLaunch& L, int k, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  if (k < 0) {
    if (cplx) hipLaunchKernelGGL(kb_chol_diag0<cd>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys);
    else hipLaunchKernelGGL(kb_chol_diag0<double>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys);
  } else {
    if (cplx)
      hipLaunchKernelGGL(kb_chol_step<cd>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys, k);
    else
      hipLaunchKernelGGL(kb_chol_step<double>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys, k);
  }
  return hipGetLastError();
}

// ---- condition estimate of a triangular factor -----------------------------
// sigma_max(T)^2 for an upper triangular FP64 T by power steps on T T*: from a
// fixed unit start vector v, each step forms u = T (T* v) and records
// ||u||, then v = u / ||u||.  The recorded norms increase towards
// sigma_max(T)^2 from below (every record is a lower bound), so
// sqrt(record_X * record_R) for X = R^{-1} bounds cond(R) from below.
namespace {
template <typename W> __device__ inline W pw_start(int64_t i) {
  // a Weyl sequence: no fixed relation to any matrix's singular vectors
  const uint64_t a = (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
  const uint64_t b = (uint64_t)(i + 1) * 0xD1B54A32D192ED03ull;
  return vmake<W>((double)(a >> 11) * 0x1.0p-53 - 0.5, (double)(b >> 11) * 0x1.0p-53 - 0.5);
}

// Two matrices (T0, T1) advance together: blockIdx.y (or the workgroup
// index for the norm) selects the matrix; vectors of matrix t sit at v + t m.
struct PwPair {
  const void* T[2];
  int64_t ld[2];
};

template <typename W>
__global__ void __launch_bounds__(256) k_pw_init(int64_t m, W* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < m) v[i] = v[m + i] = pw_start<W>(i);
}

// g_j = sum_{i <= j} conj(T_ij) v_i: a wave per column, four columns per
// workgroup.  grid (ceil(m / 4), 2), 256 threads.
template <typename W>
__global__ void __launch_bounds__(256) k_pw_adj(PwPair P, int64_t m, const W* __restrict__ v, W* __restrict__ g) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= m) return;
  const W* col = reinterpret_cast<const W*>(P.T[t]) + j * P.ld[t];
  const W* vt = v + t * m;
  W a0 = vzero<W>(), a1 = vzero<W>();
  int64_t i = lane;
  for (; i + 64 <= j; i += 128) {
    a0 = vcfma(col[i], vt[i], a0);
    a1 = vcfma(col[i + 64], vt[i + 64], a1);
  }
  if (i <= j) a0 = vcfma(col[i], vt[i], a0);
  const W a = wave_sum(vadd(a0, a1));
  if (lane == 0) g[t * m + j] = a;
}

// u_i = sum_{j >= i} T_ij g_j, one 64-row block and one chunk of cw columns
// per workgroup: lane = row, the eight waves take every eighth column of the
// chunk (each load a contiguous 64-entry piece of a column), then the waves'
// sums are added in wave order into the chunk's partial u_part[t][chunk][row]
// (zero for a chunk left of the block's diagonal).  grid (ceil(m / 64),
// chunks, 2), 512 threads.  The chunk width pw_cols(m) gives small m enough
// workgroups and large m few partials.
__host__ __device__ inline int64_t pw_cols(int64_t m) { return m <= 1024 ? 64 : (m <= 4096 ? 256 : 512); }

template <typename W>
__global__ void __launch_bounds__(512) k_pw_fwd(PwPair P, int64_t m, const W* __restrict__ g, W* __restrict__ upart) {
  const int64_t cw = pw_cols(m);
  __shared__ W part[8][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int t = blockIdx.z;
  const W* T = reinterpret_cast<const W*>(P.T[t]);
  const int64_t ldt = P.ld[t];
  const W* gt = g + t * m;
  const int64_t r0 = (int64_t)blockIdx.x * 64, r = r0 + lane;
  const int64_t jb = (int64_t)blockIdx.y * cw;
  const int64_t je = jb + cw < m ? jb + cw : m;
  W a0 = vzero<W>(), a1 = vzero<W>();
  int64_t j = (jb > r0 ? jb : r0) + wv;
  for (; j + 8 < je; j += 16) {
    if (r <= j) a0 = vfma(T[r + j * ldt], gt[j], a0);
    if (r <= j + 8) a1 = vfma(T[r + (j + 8) * ldt], gt[j + 8], a1);
  }
  if (j < je && r <= j) a0 = vfma(T[r + j * ldt], gt[j], a0);
  part[wv][lane] = vadd(a0, a1);
  __syncthreads();
  if (wv == 0 && r < m) {
    W a = part[0][lane];
#pragma unroll
    for (int w = 1; w < 8; ++w) a = vadd(a, part[w][lane]);
    upart[((int64_t)t * gridDim.y + blockIdx.y) * m + r] = a;
  }
}

// workgroup t: u_t = the sum of its chunk partials (in chunk order);
// out[t * stride + slot] = ||u_t|| (slot >= 0), v_t = u_t / ||u_t|| when the
// norm is positive and finite (else v_t keeps its entries).  grid 2, 1024
// threads.  With chunks = 0, u_t = upart_t itself (one vector).
template <typename W>
__global__ void __launch_bounds__(1024) k_pw_norm(const W* __restrict__ upart, int chunks, int64_t m,
                                                  W* __restrict__ v, double* __restrict__ out, int stride, int slot) {
  __shared__ double red[16];
  const int t = blockIdx.x;
  const int nc = chunks > 0 ? chunks : 1;
  const W* ut = upart + (int64_t)t * nc * m;
  W* vt = v + t * m;
  auto u_at = [&](int64_t i) {
    W a = ut[i];
    for (int c = 1; c < nc; ++c) a = vadd(a, ut[(int64_t)c * m + i]);
    return a;
  };
  double s2 = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 1024) s2 += vabs2(u_at(i));
  const double s = sqrt(block_sum(s2, red));
  if (threadIdx.x == 0 && slot >= 0) out[t * stride + slot] = s;
  if (!(s > 0.0) || !isfinite(s)) return;
  const double rs = 1.0 / s;
  for (int64_t i = threadIdx.x; i < m; i += 1024) vt[i] = vscale(u_at(i), rs);
}

template <typename W>
hipError_t power_t(const PwPair& P, int64_t m, void* work, double* out, int steps, hipStream_t st) {
  const int nch = (int)ceil_div(m, pw_cols(m));
  W* v = reinterpret_cast<W*>(work);
  W* g = v + 2 * m;
  W* up = v + 4 * m;
  hipLaunchKernelGGL((k_pw_init<W>), dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, m, v);
  hipLaunchKernelGGL((k_pw_norm<W>), dim3(2), dim3(1024), 0, st, v, 0, m, v, out, steps, -1);
  for (int k = 0; k < steps; ++k) {
    hipLaunchKernelGGL((k_pw_adj<W>), dim3((unsigned)ceil_div(m, 4), 2), dim3(256), 0, st, P, m, v, g);
    hipLaunchKernelGGL((k_pw_fwd<W>), dim3((unsigned)ceil_div(m, 64), (unsigned)nch, 2), dim3(512), 0, st, P, m, g,
                       up);
    hipLaunchKernelGGL((k_pw_norm<W>), dim3(2), dim3(1024), 0, st, up, nch, m, v, out, steps, k);
  }
  return hipGetLastError();
}
}  // namespace

int64_t power_work_elems(int64_t m) { return (4 + 2 * ceil_div(m, pw_cols(m))) * m; }

hipError_t launch_power_sq(bool cplx, const void* T0, int64_t ld0, const void* T1, int64_t ld1, int64_t m, void* work,
                           double* out, int steps, hipStream_t st) {
  if (m < 1 || ld0 < m || ld1 < m || steps < 1) return hipErrorInvalidValue;
  PwPair P;
  P.T[0] = T0;
  P.T[1] = T1;
  P.ld[0] = ld0;
  P.ld[1] = ld1;
  return cplx ? power_t<cd>(P, m, work, out, steps, st) : power_t<double>(P, m, work, out, steps, st);
}

namespace {
// sigma_max(T)^2 record after `steps` power steps on T T* (T upper, FP64,
// ld ldt), the same steps as launch_power_sq, inside one workgroup of
// kBPowT threads: g = T* v a wave per column, u = T g a 64-row block at a
// time (lane = row, the waves taking every kBPowW-th column).
constexpr int kBPowT = 1024, kBPowW = kBPowT / 64;

template <typename W>
__device__ double b_power_one(const W* __restrict__ T, int64_t ldt, int64_t m, W* v, W* g, W* u, int steps,
                              double* red, W (*part)[64]) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int64_t i = t; i < m; i += kBPowT) v[i] = pw_start<W>(i);
  __syncthreads();
  double s2 = 0.0;
  for (int64_t i = t; i < m; i += kBPowT) s2 += vabs2(v[i]);
  const double nrm = sqrt(block_sum(s2, red));
  for (int64_t i = t; i < m; i += kBPowT) v[i] = vscale(v[i], 1.0 / nrm);
  double rec = 0.0;
  for (int k = 0; k < steps; ++k) {
    __syncthreads();
    for (int64_t j = wv; j < m; j += kBPowW) {
      W a = vzero<W>();
      for (int64_t i = lane; i <= j; i += 64) a = vcfma(T[i + j * ldt], v[i], a);
      a = wave_sum(a);
      if (lane == 0) g[j] = a;
    }
    __syncthreads();
    s2 = 0.0;
    for (int64_t r0 = 0; r0 < m; r0 += 64) {
      const int64_t r = r0 + lane;
      W a0 = vzero<W>(), a1 = vzero<W>();
      int64_t j = r0 + wv;
      for (; j + kBPowW < m; j += 2 * kBPowW) {
        if (r <= j) a0 = vfma(T[r + j * ldt], g[j], a0);
        if (r <= j + kBPowW) a1 = vfma(T[r + (j + kBPowW) * ldt], g[j + kBPowW], a1);
      }
      if (j < m && r <= j) a0 = vfma(T[r + j * ldt], g[j], a0);
      part[wv][lane] = vadd(a0, a1);
      __syncthreads();
      if (wv == 0 && r < m) {
        W a = part[0][lane];
        for (int w = 1; w < kBPowW; ++w) a = vadd(a, part[w][lane]);
        u[r] = a;
        s2 += vabs2(a);
      }
      __syncthreads();
    }
    rec = sqrt(block_sum(s2, red));
    if (!(rec > 0.0) || !isfinite(rec)) return rec;
    for (int64_t i = t; i < m; i += kBPowT) v[i] = vscale(u[i], 1.0 / rec);
  }
  return rec;
}

template <typename W>
__global__ void __launch_bounds__(kBPowT) kb_power(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                   int nsys, int steps) {
  __shared__ double red[kBPowW];
  __shared__ W part[kBPowW][64];
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  const int64_t m = s.m;
  W* v = reinterpret_cast<W*>(s.pw);
  const double pr = b_power_one<W>(reinterpret_cast<const W*>(s.R), m, m, v, v + m, v + 2 * m, steps, red, part);
  __syncthreads();
  const double px =
      b_power_one<W>(reinterpret_cast<const W*>(s.X), s.ldx, m, v, v + m, v + 2 * m, steps, red, part);
  if (threadIdx.x == 0) s.diag[3] = pr * px;
}
}  // namespace

hipError_t launch_b_power(bool cplx, const BLaunch& L, int steps, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  if (cplx)
    hipLaunchKernelGGL(kb_power<cd>, dim3((unsigned)L.total), dim3(kBPowT), 0, st, L.sys, L.grid, L.nsys, steps);
  else
    hipLaunchKernelGGL(kb_power<double>, dim3((unsigned)L.total), dim3(kBPowT), 0, st, L.sys, L.grid, L.nsys, steps);
  return hipGetLastError();
}

}  // namespace mn
