// R with R* R = G for the Hermitian positive definite Gram matrix G = S* S of
// the sketch (Section 4, Step 2 uses only the triangular factor of S: R* R =
// S* S holds for the R of any QR decomposition S = Q R).
//
// Right-looking blocked Cholesky on 32 x 32 tiles, one launch per block step
// k: every workgroup factors the diagonal tile G_kk itself (32 steps in LDS),
// then
//   tile (k, j), j >= k:        R_kj = R_kk^{-*} G_kj      (written to R)
//   tile (i, j), k < i <= j:    G_ij -= R_ki^* R_kj        (Schur complement)
// recomputing the R_k* tiles it needs.  G tiles of block row k are only read
// during step k, so R goes to a separate buffer and no step races with
// itself.  FP64 throughout.
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
// T = R* R.  Padding rows/columns beyond `valid` are set to the identity so
// the factor stays invertible.  One barrier per column: the trailing update
// uses the unscaled row c divided by the pivot, rows are scaled at the end.
// Returns false if a pivot is not positive and finite.
template <typename V>
__device__ bool chol_tile(V* T, int valid, double* piv) {
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
    const int r = e % CB, c = e / CB;
    if (r >= valid || c >= valid) T[r + c * LDC] = (r == c) ? vmake<V>(1.0, 0.0) : vzero<V>();
  }
  __syncthreads();
  for (int c = 0; c < CB; ++c) {
    const double d = vre(T[c + c * LDC]);
    if (threadIdx.x == 0) piv[c] = d;
    const double inv = 1.0 / d;
    for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
      const int i = e % CB, j = e / CB;
      if (i > c && i <= j) T[i + j * LDC] = vsub(T[i + j * LDC], vscale(vcmul(T[c + i * LDC], T[c + j * LDC]), inv));
    }
    __syncthreads();
  }
  bool ok = true;
  for (int c = 0; c < CB; ++c) ok = ok && (piv[c] > 0.0) && isfinite(piv[c]);
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
    const int i = e % CB, j = e / CB;
    const double s = piv[i] > 0.0 ? 1.0 / sqrt(piv[i]) : 0.0;
    if (i < j) T[i + j * LDC] = vscale(T[i + j * LDC], s);
    else if (i == j) T[i + j * LDC] = vmake<V>(piv[i] > 0.0 ? sqrt(piv[i]) : 0.0, 0.0);
    else T[i + j * LDC] = vzero<V>();
  }
  __syncthreads();
  return ok;
}

// In place: B1 <- R^{-*} B1 and (if B2) B2 <- R^{-*} B2 (forward substitution
// on R* X = B, R upper).  One wave; lane j takes column j of B1 (lanes 0-31)
// or of B2 (lanes 32-63) in registers, so the 32 dependent row steps need no
// barrier: every lane reads the same entries of R (LDS broadcast).
template <typename V>
__device__ void solve_tiles(const V* R, V* B1, V* B2) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    V* B = lane < CB ? B1 : B2;
    const int j = lane & (CB - 1);
    if (B) {
      V x[CB];
#pragma unroll
      for (int r = 0; r < CB; ++r) x[r] = B[r + j * LDC];
#pragma unroll
      for (int q = 0; q < CB; ++q) {
        x[q] = vscale(x[q], 1.0 / vre(R[q + q * LDC]));
#pragma unroll
        for (int r = q + 1; r < CB; ++r) x[r] = vsub(x[r], vcmul(R[q + r * LDC], x[q]));
      }
#pragma unroll
      for (int r = 0; r < CB; ++r) B[r + j * LDC] = x[r];
    }
  }
  __syncthreads();
}

// T <- A^* B for 32 x 32 tiles in LDS (C may alias neither)
template <typename V>
__device__ void tile_ahb(const V* A, const V* B, V* C) {
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
    const int r = e % CB, c = e / CB;
    V acc = vzero<V>();
#pragma unroll 8
    for (int q = 0; q < CB; ++q) acc = vcfma(A[q + r * LDC], B[q + c * LDC], acc);
    C[r + c * LDC] = acc;
  }
}
// T <- Y B for tiles in LDS (Y = R_kk^{-*}, lower triangular)
template <typename V>
__device__ void tile_ab_lower(const V* Y, const V* B, V* C) {
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
    const int r = e % CB, c = e / CB;
    V acc = vzero<V>();
    for (int q = 0; q <= r; ++q) acc = vfma(Y[r + q * LDC], B[q + c * LDC], acc);
    C[r + c * LDC] = acc;
  }
}

// Factor the (updated) diagonal tile held in T for block k: R_kk -> R,
// Y_kk = R_kk^{-*} -> Yd[k] (32 x 32, column-major, ld 32).
template <typename V>
__device__ void finish_diag(V* T, V* Y, double* piv, int k, int64_t m, V* R, int64_t ldr, V* Yd, int32_t* bad) {
  const int valid = (int)((m - (int64_t)k * CB) < CB ? (m - (int64_t)k * CB) : CB);
  const bool ok = chol_tile(T, valid, piv);
  if (!ok && threadIdx.x == 0) bad[0] = 1;
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
    const int r = e % CB, c = e / CB;
    Y[r + c * LDC] = (r == c) ? vmake<V>(1.0, 0.0) : vzero<V>();
  }
  __syncthreads();
  solve_tiles(T, Y, (V*)nullptr);  // Y = R_kk^{-*}
  V* yd = Yd + (int64_t)k * CB * CB;
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
    const int r = e % CB, c = e / CB;
    const int64_t gr = (int64_t)k * CB + r, gc = (int64_t)k * CB + c;
    if (gr < m && gc < m) R[gr + gc * ldr] = T[r + c * LDC];
    yd[e] = Y[r + c * LDC];
  }
  // the strictly lower part of R's block column k
  const int64_t below = m - (int64_t)(k + 1) * CB;
  for (int64_t e = threadIdx.x; e < below * CB; e += blockDim.x) {
    const int64_t r = (int64_t)(k + 1) * CB + e % below;
    const int64_t c = (int64_t)k * CB + e / below;
    if (c < m) R[r + c * ldr] = vzero<V>();
  }
}

// Block step 0's diagonal tile (one workgroup).
template <typename V>
__device__ __forceinline__ void k_chol_diag0_body(const Bk bk, V* __restrict__ G, int64_t ldg, int64_t m,
                                                   V* __restrict__ R, int64_t ldr, V* __restrict__ Yd,
                                                   int32_t* __restrict__ bad) {
  (void)bk;
  __shared__ V T[CB * LDC];
  __shared__ V Y[CB * LDC];
  __shared__ double piv[CB];
  tile_in(T, G, ldg, m, 0, 0);
  __syncthreads();
  finish_diag(T, Y, piv, 0, m, R, ldr, Yd, bad);
}
template <typename V>
__global__ void __launch_bounds__(256) k_chol_diag0(V* __restrict__ G, int64_t ldg, int64_t m, V* __restrict__ R,
                                                    int64_t ldr, V* __restrict__ Yd, int32_t* __restrict__ bad) {
  k_chol_diag0_body<V>(bk_hw(), G, ldg, m, R, ldr, Yd, bad);
}

// Block step k (R_kk and Y_kk = R_kk^{-*} known):
//   tile (k, j), j > k:      R_kj = Y_kk G_kj                     -> R
//   tile (i, j), k < i <= j: G_ij -= (Y_kk G_ki)^* (Y_kk G_kj); the workgroup
//                            of (k+1, k+1) then factors it (R, Y of block k+1).
// grid = (nbk - k - 1) + (nbk - k - 1)(nbk - k)/2 workgroups.
template <typename V>
__device__ __forceinline__ void k_chol_step_body(const Bk bk, V* __restrict__ G, int64_t ldg, int64_t m, int k, int nbk,
                                                   V* __restrict__ R, int64_t ldr, V* __restrict__ Yd,
                                                   int32_t* __restrict__ bad) {
  __shared__ V Y[CB * LDC];
  __shared__ V T1[CB * LDC];
  __shared__ V T2[CB * LDC];
  __shared__ V T3[CB * LDC];
  __shared__ double piv[CB];
  const int nrow = nbk - k - 1;
  int bi, bj;
  int w = bk.x;
  if (w < nrow) {
    bi = k;
    bj = k + 1 + w;
  } else {
    w -= nrow;
    bi = k + 1;
    int len = nbk - bi;
    while (w >= len) {
      w -= len;
      ++bi;
      len = nbk - bi;
    }
    bj = bi + w;
  }
  const V* yd = Yd + (int64_t)k * CB * CB;
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) Y[(e % CB) + (e / CB) * LDC] = yd[e];
  if (bi == k) {
    tile_in(T1, G, ldg, m, k, bj);
    __syncthreads();
    tile_ab_lower(Y, T1, T2);  // R_kj
    __syncthreads();
    for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
      const int r = e % CB, c = e / CB;
      const int64_t gr = (int64_t)k * CB + r, gc = (int64_t)bj * CB + c;
      if (gr < m && gc < m) R[gr + gc * ldr] = T2[r + c * LDC];
    }
    return;
  }
  // trailing tile: R_ki (T2), R_kj (T3), then G_ij -= R_ki^* R_kj
  tile_in(T1, G, ldg, m, k, bi);
  __syncthreads();
  tile_ab_lower(Y, T1, T2);
  __syncthreads();
  if (bj != bi) {
    tile_in(T1, G, ldg, m, k, bj);
    __syncthreads();
    tile_ab_lower(Y, T1, T3);
    __syncthreads();
  }
  const V* Rj = bj != bi ? T3 : T2;
  tile_in(T1, G, ldg, m, bi, bj);
  __syncthreads();
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
    const int r = e % CB, c = e / CB;
    V acc = vzero<V>();
#pragma unroll 8
    for (int q = 0; q < CB; ++q) acc = vcfma(T2[q + r * LDC], Rj[q + c * LDC], acc);
    T1[r + c * LDC] = vsub(T1[r + c * LDC], acc);
  }
  __syncthreads();
  if (bi == k + 1 && bj == k + 1) {
    // the next diagonal tile is final: factor it for block step k + 1
    finish_diag(T1, T3, piv, k + 1, m, R, ldr, Yd, bad);
    return;
  }
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
    const int r = e % CB, c = e / CB;
    const int64_t gr = (int64_t)bi * CB + r, gc = (int64_t)bj * CB + c;
    if (gr < m && gc < m && gr <= gc) G[gr + gc * ldg] = T1[r + c * LDC];
  }
}
template <typename V>
__global__ void __launch_bounds__(256) k_chol_step(V* __restrict__ G, int64_t ldg, int64_t m, int k, int nbk,
                                                   V* __restrict__ R, int64_t ldr, V* __restrict__ Yd,
                                                   int32_t* __restrict__ bad) {
  k_chol_step_body<V>(bk_hw(), G, ldg, m, k, nbk, R, ldr, Yd, bad);
}

template <typename V>
hipError_t chol_impl(void* G, int64_t ldg, int64_t m, void* R, int64_t ldr, void* Yd, int32_t* bad, hipStream_t st) {
  const int nbk = (int)ceil_div(m, CB);
  hipLaunchKernelGGL((k_chol_diag0<V>), dim3(1), dim3(256), 0, st, reinterpret_cast<V*>(G), ldg, m,
                     reinterpret_cast<V*>(R), ldr, reinterpret_cast<V*>(Yd), bad);
  for (int k = 0; k + 1 < nbk; ++k) {
    const int nrow = nbk - k - 1;
    const int ntrail = (nbk - k - 1) * (nbk - k) / 2;
    hipLaunchKernelGGL((k_chol_step<V>), dim3((unsigned)(nrow + ntrail)), dim3(256), 0, st, reinterpret_cast<V*>(G),
                       ldg, m, k, nbk, reinterpret_cast<V*>(R), ldr, reinterpret_cast<V*>(Yd), bad);
  }
  return hipGetLastError();
}

}  // namespace

int64_t chol_scratch_elems(int64_t m) { return ceil_div(m, CB) * CB * CB; }

hipError_t launch_chol(bool cplx, void* G, int64_t ldg, int64_t m, void* R, int64_t ldr, void* Yd, int32_t* bad,
                       hipStream_t st) {
  if (m < 1 || ldg < m || ldr < m) return hipErrorInvalidValue;
  return cplx ? chol_impl<cd>(G, ldg, m, R, ldr, Yd, bad, st) : chol_impl<double>(G, ldg, m, R, ldr, Yd, bad, st);
}

namespace {
template <typename V>
__global__ void __launch_bounds__(256) kb_chol_diag0(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                     int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_chol_diag0_body<V>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<V*>(s.G), s.m, s.m,
                       reinterpret_cast<V*>(s.R), s.m, reinterpret_cast<V*>(s.Yd), s.flags + 1);
}
template <typename V>
__global__ void __launch_bounds__(256) kb_chol_step(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                    int nsys, int k) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_chol_step_body<V>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<V*>(s.G), s.m, s.m, k,
                      (int)ceil_div(s.m, CB), reinterpret_cast<V*>(s.R), s.m, reinterpret_cast<V*>(s.Yd),
                      s.flags + 1);
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

}  // namespace mn
