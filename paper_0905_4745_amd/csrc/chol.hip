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

template <typename V>
__device__ __forceinline__ void k_chol_step_body(const Bk bk, V* __restrict__ G, int64_t ldg, int64_t m, int k, int nbk,
                                                   V* __restrict__ R, int64_t ldr, int32_t* __restrict__ bad) {
  __shared__ V Rkk[CB * LDC];
  __shared__ V T1[CB * LDC];
  __shared__ V T2[CB * LDC];
  __shared__ double piv[CB];
  // workgroup -> tile: first the nbk - k tiles of block row k, then the
  // trailing upper tiles (i, j), k < i <= j, row by row
  const int nrow = nbk - k;
  int bi, bj;
  int w = bk.x;
  if (w < nrow) {
    bi = k;
    bj = k + w;
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
  const int valid = (int)((m - (int64_t)k * CB) < CB ? (m - (int64_t)k * CB) : CB);
  tile_in(Rkk, G, ldg, m, k, k);
  __syncthreads();
  const bool ok = chol_tile(Rkk, valid, piv);
  if (bi == k) {
    if (bj == k) {
      if (!ok && threadIdx.x == 0) bad[0] = 1;
      for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
        const int r = e % CB, c = e / CB;
        const int64_t gr = (int64_t)k * CB + r, gc = (int64_t)k * CB + c;
        if (gr < m && gc < m) R[gr + gc * ldr] = Rkk[r + c * LDC];
      }
      // zero the strictly lower part of R's block column k below the diagonal tile
      for (int64_t e = threadIdx.x; e < (m - (int64_t)(k + 1) * CB) * CB; e += blockDim.x) {
        const int64_t r = (int64_t)(k + 1) * CB + e % (m - (int64_t)(k + 1) * CB);
        const int64_t c = (int64_t)k * CB + e / (m - (int64_t)(k + 1) * CB);
        if (r < m && c < m) R[r + c * ldr] = vzero<V>();
      }
      return;
    }
    tile_in(T1, G, ldg, m, k, bj);
    __syncthreads();
    solve_tiles(Rkk, T1, (V*)nullptr);
    for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
      const int r = e % CB, c = e / CB;
      const int64_t gr = (int64_t)k * CB + r, gc = (int64_t)bj * CB + c;
      if (gr < m && gc < m) R[gr + gc * ldr] = T1[r + c * LDC];
    }
    // R's strictly lower tile (bj, k) is zero
    for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
      const int r = e % CB, c = e / CB;
      const int64_t gr = (int64_t)bj * CB + r, gc = (int64_t)k * CB + c;
      if (gr < m && gc < m) R[gr + gc * ldr] = vzero<V>();
    }
    return;
  }
  // trailing tile: R_ki and R_kj, then G_ij -= R_ki^* R_kj
  tile_in(T1, G, ldg, m, k, bi);
  if (bj != bi) tile_in(T2, G, ldg, m, k, bj);
  __syncthreads();
  solve_tiles(Rkk, T1, bj != bi ? T2 : (V*)nullptr);
  const V* Rj = bj != bi ? T2 : T1;
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
    const int r = e % CB, c = e / CB;
    const int64_t gr = (int64_t)bi * CB + r, gc = (int64_t)bj * CB + c;
    if (gr >= m || gc >= m || gr > gc) continue;
    V acc = vzero<V>();
    for (int q = 0; q < CB; ++q) acc = vcfma(T1[q + r * LDC], Rj[q + c * LDC], acc);
    G[gr + gc * ldg] = vsub(G[gr + gc * ldg], acc);
  }
}
template <typename V>
__global__ void __launch_bounds__(256) k_chol_step(V* __restrict__ G, int64_t ldg, int64_t m, int k, int nbk,
                                                   V* __restrict__ R, int64_t ldr, int32_t* __restrict__ bad) {
  k_chol_step_body<V>(bk_hw(), G, ldg, m, k, nbk, R, ldr, bad);
}

template <typename V>
hipError_t chol_impl(void* G, int64_t ldg, int64_t m, void* R, int64_t ldr, int32_t* bad, hipStream_t st) {
  const int nbk = (int)ceil_div(m, CB);
  for (int k = 0; k < nbk; ++k) {
    const int nrow = nbk - k;
    const int ntrail = (nbk - k - 1) * (nbk - k) / 2;
    hipLaunchKernelGGL((k_chol_step<V>), dim3((unsigned)(nrow + ntrail)), dim3(256), 0, st, reinterpret_cast<V*>(G),
                       ldg, m, k, nbk, reinterpret_cast<V*>(R), ldr, bad);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_chol(bool cplx, void* G, int64_t ldg, int64_t m, void* R, int64_t ldr, int32_t* bad,
                       hipStream_t st) {
  if (m < 1 || ldg < m || ldr < m) return hipErrorInvalidValue;
  return cplx ? chol_impl<cd>(G, ldg, m, R, ldr, bad, st) : chol_impl<double>(G, ldg, m, R, ldr, bad, st);
}

namespace {
template <typename V>
__global__ void __launch_bounds__(256) kb_chol_step(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                    int nsys, int k) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_chol_step_body<V>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<V*>(s.G), s.m, s.m, k,
                      (int)ceil_div(s.m, CB), reinterpret_cast<V*>(s.R), s.m, s.flags + 1);
}
}  // namespace

// one block step of every system that has block column k (grid: as launch_chol's step k)
hipError_t launch_b_chol_step(bool cplx, const BLaunch& L, int k, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  if (cplx) hipLaunchKernelGGL(kb_chol_step<cd>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys, k);
  else hipLaunchKernelGGL(kb_chol_step<double>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys, k);
  return hipGetLastError();
}

}  // namespace mn
