// Steps 2-3 of the method made explicit (Section 4, eqs. lineq and
// nonminnorm), a check and export path beside the solve, which folds them
// into Step 4:
//   g = R^{-*} b,  u = R^{-1} g,  z = S u   (the minimal-norm solution of
//   S* z = b: z = Q_S R^{-*} b with S = Q_S R, eq. lineq)
//   c = T* z = D* F* S* z                    (eq. nonminnorm)
// With X = R^{-1} (FP64, upper, from the factorisation): g = X* b, u = X g.
// S* z scatters z to the kept rows; F* y = conj(F conj(y)) is computed by
// the sketch kernels on one row (d = 1, every output kept); c = conj(d) o
// conj(that) for complex data, d o (Hartley transform of y) for real data.
// Lemma 5.1 gives A c = b; the residual is computed in FP64 on the device.
#include "common.hpp"
#include "kernels.hpp"

namespace mn {

// g_j = sum_{i <= j} conj(X_ij) b_i: one wave per column of X.  grid m, 64 threads.
template <typename W>
__global__ void __launch_bounds__(64) k_st_xhb(const W* __restrict__ X, int64_t ldx, int64_t m,
                                               const W* __restrict__ b, W* __restrict__ g) {
  const int64_t j = blockIdx.x;
  W a = vzero<W>();
  for (int64_t i = threadIdx.x; i <= j; i += 64) a = vcfma(X[i + j * ldx], b[i], a);
  a = wave_sum(a);
  if (threadIdx.x == 0) g[j] = a;
}

// u_i = sum_{j >= i} X_ij g_j: one thread per row (consecutive threads read
// consecutive entries of each column).  grid ceil(m / 256), 256 threads.
template <typename W>
__global__ void __launch_bounds__(256) k_st_xg(const W* __restrict__ X, int64_t ldx, int64_t m,
                                               const W* __restrict__ g, W* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  W a = vzero<W>();
  for (int64_t j = i; j < m; ++j) a = vfma(X[i + j * ldx], g[j], a);
  u[i] = a;
}

// z_k = sum_i S(k, i) u_i (S column-major l x m in the data's precision,
// promoted); y[idx[k]] = z_k (y zeroed before).  grid ceil(l / 256), 256 threads.
template <typename V, typename W>
__global__ void __launch_bounds__(256) k_st_z(const V* __restrict__ S, int64_t lds, int64_t l, int64_t m,
                                              const W* __restrict__ u, const int32_t* __restrict__ idx,
                                              W* __restrict__ z, W* __restrict__ y) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= l) return;
  W a = vzero<W>();
  for (int64_t i = 0; i < m; ++i) a = vfma(vconv<W>(S[k + i * lds]), u[i], a);
  z[k] = a;
  y[idx[k]] = a;
}

// d' = 1 and idx' = 0 .. N-1 (the one-row transform that keeps every output)
template <typename W>
__global__ void __launch_bounds__(256) k_st_ones_iota(int64_t N, W* __restrict__ ones, int32_t* __restrict__ iota) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  ones[j] = vmake<W>(1.0, 0.0);
  iota[j] = (int32_t)j;
}

// c_j = conj(d_j) conj(t_j) with t = F conj(y) (complex), or d_j t_j with t
// the Hartley transform of y (real).  grid ceil(N / 256), 256 threads.
template <typename W>
__global__ void __launch_bounds__(256) k_st_c(const W* __restrict__ t, const W* __restrict__ d, int64_t N,
                                              W* __restrict__ c) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  if constexpr (VT<W>::cplx) c[j] = vconj(vmul(d[j], t[j]));
  else c[j] = d[j] * t[j];
}

// out[0] = ||b - sum of the chunk partials||^2, out[1] = ||b||^2 (one
// workgroup; chunks = 0: no partials, out[0] = out[1] = ||b||^2)
template <typename W>
__global__ void __launch_bounds__(256) k_st_resid(const W* __restrict__ qpart, int chunks, int64_t m,
                                                  const W* __restrict__ b, double* __restrict__ out) {
  __shared__ double red[4];
  double r2 = 0.0, b2 = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    W q = vzero<W>();
    for (int k = 0; k < chunks; ++k) q = vadd(q, qpart[(int64_t)k * m + i]);
    r2 += vabs2(vsub(b[i], q));
    b2 += vabs2(b[i]);
  }
  r2 = block_sum(r2, red);
  b2 = block_sum(b2, red);
  if (threadIdx.x == 0) {
    out[0] = r2;
    out[1] = b2;
  }
}

template <typename W>
static hipError_t st_solve_t(const void* X, int64_t ldx, int64_t m, const void* b, void* g, void* u, hipStream_t st) {
  const W* Xw = reinterpret_cast<const W*>(X);
  hipLaunchKernelGGL((k_st_xhb<W>), dim3((unsigned)m), dim3(64), 0, st, Xw, ldx, m, reinterpret_cast<const W*>(b),
                     reinterpret_cast<W*>(g));
  hipLaunchKernelGGL((k_st_xg<W>), dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, Xw, ldx, m,
                     reinterpret_cast<const W*>(g), reinterpret_cast<W*>(u));
  return hipGetLastError();
}

hipError_t launch_st_solve(bool cplx, const void* X, int64_t ldx, int64_t m, const void* b, void* g, void* u,
                           hipStream_t st) {
  return cplx ? st_solve_t<cd>(X, ldx, m, b, g, u, st) : st_solve_t<double>(X, ldx, m, b, g, u, st);
}

hipError_t launch_st_z(int dtype, const void* S, int64_t lds, int64_t l, int64_t m, const void* u, const int32_t* idx,
                       void* z, void* y, hipStream_t st) {
  const dim3 grid((unsigned)ceil_div(l, 256));
  switch (dtype) {
    case 0: hipLaunchKernelGGL((k_st_z<cd, cd>), grid, dim3(256), 0, st, (const cd*)S, lds, l, m, (const cd*)u, idx,
                               (cd*)z, (cd*)y); break;
    case 1: hipLaunchKernelGGL((k_st_z<cf, cd>), grid, dim3(256), 0, st, (const cf*)S, lds, l, m, (const cd*)u, idx,
                               (cd*)z, (cd*)y); break;
    case 2: hipLaunchKernelGGL((k_st_z<double, double>), grid, dim3(256), 0, st, (const double*)S, lds, l, m,
                               (const double*)u, idx, (double*)z, (double*)y); break;
    case 3: hipLaunchKernelGGL((k_st_z<float, double>), grid, dim3(256), 0, st, (const float*)S, lds, l, m,
                               (const double*)u, idx, (double*)z, (double*)y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_st_ones_iota(bool cplx, int64_t N, void* ones, int32_t* iota, hipStream_t st) {
  const dim3 grid((unsigned)ceil_div(N, 256));
  if (cplx) hipLaunchKernelGGL((k_st_ones_iota<cd>), grid, dim3(256), 0, st, N, (cd*)ones, iota);
  else hipLaunchKernelGGL((k_st_ones_iota<double>), grid, dim3(256), 0, st, N, (double*)ones, iota);
  return hipGetLastError();
}

hipError_t launch_st_c(bool cplx, const void* t, const void* d, int64_t N, void* c, hipStream_t st) {
  const dim3 grid((unsigned)ceil_div(N, 256));
  if (cplx) hipLaunchKernelGGL((k_st_c<cd>), grid, dim3(256), 0, st, (const cd*)t, (const cd*)d, N, (cd*)c);
  else hipLaunchKernelGGL((k_st_c<double>), grid, dim3(256), 0, st, (const double*)t, (const double*)d, N, (double*)c);
  return hipGetLastError();
}

hipError_t launch_st_resid(bool cplx, const void* qpart, int chunks, int64_t m, const void* b, double* out,
                           hipStream_t st) {
  if (cplx)
    hipLaunchKernelGGL((k_st_resid<cd>), dim3(1), dim3(256), 0, st, (const cd*)qpart, chunks, m, (const cd*)b, out);
  else
    hipLaunchKernelGGL((k_st_resid<double>), dim3(1), dim3(256), 0, st, (const double*)qpart, chunks, m,
                       (const double*)b, out);
  return hipGetLastError();
}

}  // namespace mn
