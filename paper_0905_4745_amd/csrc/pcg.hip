// Step 4 of the method read as preconditioned conjugate gradients on
// A A* y = b (A c = b by Lemma 5.1 makes these the normal equations of
// eq. overdet), preconditioned by R* R with R from Step 2's factorisation.
//
// The m-vectors of the iteration (y, r, p, z, s, q) are FP64 whatever the
// precision of A; their inner products and norms, and the stopping test,
// are FP64 too.  The preconditioner solves R* s = r and R z = s run in FP64
// on R promoted from its storage precision, blocked by 32 x 32 diagonal
// blocks whose inverses are formed once (k_inv_diag); R stays in cache.
//
// Stopping rules, with rho = ||R^{-*} r||^2 and xi = Re(y^*(b - r)) = ||A* y||^2
// (||x - p||^2 <= rho since the SRFT has orthonormal rows):
//   rule 0 -- the paper's precision for Step 4, f - f* <= delta f*,
//             delta = eps^2 l / (alpha N): rho <= delta (rho0 - (sqrt xi + sqrt rho)^2)
//             (rule 1 when l = N: then f* = 0);
//   rule 1 -- ||x - p|| <= eps ||p||:  rho <= (eps / (1 + eps))^2 xi;
//   rule 2 -- relative reduction of an inner solve: rho <= eps^2 rho0.
#include "common.hpp"
#include "kernels.hpp"

namespace mn {

constexpr int TB = 32;        // triangular block
constexpr int PT = 1024;      // threads of the single-workgroup kernels

// X_k = inverse of the k-th 32 x 32 diagonal block of R (upper triangular),
// in FP64.  Ragged last block padded with the identity.  grid = K blocks.
template <typename RV, typename W>
__global__ void __launch_bounds__(256) k_inv_diag(const RV* __restrict__ R, int64_t ldr, int64_t m, W* __restrict__ X) {
  __shared__ W T[TB * TB];
  __shared__ W Xs[TB * TB];
  const int64_t c0 = (int64_t)blockIdx.x * TB;
  for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) {
    const int r = e % TB, c = e / TB;
    W v = vzero<W>();
    if (c0 + r < m && c0 + c < m) v = vconv<W>(R[(c0 + r) + (c0 + c) * ldr]);
    else if (r == c) v = vmake<W>(1.0, 0.0);
    T[e] = v;
    Xs[e] = vzero<W>();
  }
  __syncthreads();
  // column c of X solves T x = e_c by back substitution (thread c)
  if (threadIdx.x < TB) {
    const int c = threadIdx.x;
    for (int i = c; i >= 0; --i) {
      W acc = (i == c) ? vmake<W>(1.0, 0.0) : vzero<W>();
      for (int j = i + 1; j <= c; ++j) acc = vsub(acc, vmul(T[i + j * TB], Xs[j + c * TB]));
      // divide by T[i, i]
      const W d = T[i + i * TB];
      const double den = vabs2(d);
      Xs[i + c * TB] = vscale(vcmul(d, acc), 1.0 / den);  // conj(d) acc / |d|^2
    }
  }
  __syncthreads();
  W* Xo = X + (int64_t)blockIdx.x * TB * TB;
  for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) Xo[e] = Xs[e];
}

// --------------------------- triangular solves ------------------------------
// s = R^{-*} r.  All PT threads.  r, s in global memory (may alias? no).
template <typename RV, typename W>
__device__ void trsv_adj(const RV* __restrict__ R, int64_t ldr, const W* __restrict__ X, int64_t m,
                         const W* __restrict__ r, W* __restrict__ s, W* acc_sh, W* tmp_sh) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int nw = PT / 64;
  const int64_t K = ceil_div(m, TB);
  for (int64_t kb = 0; kb < K; ++kb) {
    const int64_t c0 = kb * TB;
    const int nb = (int)((m - c0) < TB ? (m - c0) : TB);
    // acc[c] = sum_{q < c0} conj(R[q, c0 + c]) s[q]
    for (int c = wv; c < TB; c += nw) {
      W part = vzero<W>();
      if (c < nb) {
        const RV* col = R + (c0 + c) * ldr;
        for (int64_t q = lane; q < c0; q += 64) part = vcfma(vconv<W>(col[q]), s[q], part);
      }
      part = wave_sum(part);
      if (lane == 0) acc_sh[c] = part;
    }
    __syncthreads();
    if (t < TB) tmp_sh[t] = (t < nb) ? vsub(r[c0 + t], acc_sh[t]) : vzero<W>();
    __syncthreads();
    if (t < nb) {
      const W* Xk = X + kb * TB * TB;
      W v = vzero<W>();
      for (int cp = 0; cp <= t; ++cp) v = vcfma(Xk[cp + t * TB], tmp_sh[cp], v);
      s[c0 + t] = v;
    }
    __syncthreads();
  }
}

// z = R^{-1} s, using tv (global, m entries) as the running right-hand side.
template <typename RV, typename W>
__device__ void trsv_fwd(const RV* __restrict__ R, int64_t ldr, const W* __restrict__ X, int64_t m,
                         const W* __restrict__ s, W* __restrict__ z, W* __restrict__ tv) {
  const int t = threadIdx.x;
  for (int64_t q = t; q < m; q += PT) tv[q] = s[q];
  __syncthreads();
  const int64_t K = ceil_div(m, TB);
  for (int64_t kb = K - 1; kb >= 0; --kb) {
    const int64_t c0 = kb * TB;
    const int nb = (int)((m - c0) < TB ? (m - c0) : TB);
    if (t < nb) {
      const W* Xk = X + kb * TB * TB;
      W v = vzero<W>();
      for (int cp = t; cp < nb; ++cp) v = vfma(Xk[t + cp * TB], tv[c0 + cp], v);
      z[c0 + t] = v;
    }
    __syncthreads();
    for (int64_t q = t; q < c0; q += PT) {
      W acc = vzero<W>();
      for (int c = 0; c < nb; ++c) acc = vfma(vconv<W>(R[q + (c0 + c) * ldr]), z[c0 + c], acc);
      tv[q] = vsub(tv[q], acc);
    }
    __syncthreads();
  }
}

template <typename W> __device__ inline double block_dot_re(const W* a, const W* b, int64_t m, double* red) {
  double p = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += PT) p += vre(vcmul(a[i], b[i]));
  return block_sum(p, red);
}

__device__ inline bool stop_test(const PcgState& st, double rho, double xi) {
  if (st.rule == 2) return rho <= st.eps * st.eps * st.rho0;
  if (st.rule == 0 && st.l < st.N) {
    const double delta = st.eps * st.eps * st.l / (st.alpha * st.N);
    const double g = sqrt(xi) + sqrt(rho);
    return rho <= delta * (st.rho0 - g * g);
  }
  const double tol = st.eps / (1.0 + st.eps);
  return rho <= tol * tol * xi;
}

// Start (or restart) CG from y = 0 with residual r = rhs:
//   r = rhs, s = R^{-*} r, z = R^{-1} s, p = z, rho0 = rho = ||s||^2.
// If parts != nullptr, rhs = b - sum_c parts[c*m + i] (an FP64 residual
// b - A A* y_outer), and the outer certificate test (rule 1 with eps_outer)
// is evaluated on it first: when it passes, the solve is marked finished.
template <typename RV, typename W>
__global__ void __launch_bounds__(PT) k_pcg_start(const RV* __restrict__ R, int64_t ldr, const W* __restrict__ X,
                                                  int64_t m, const W* __restrict__ b, const W* __restrict__ parts,
                                                  int nparts, const W* __restrict__ y_outer, W* __restrict__ y,
                                                  W* __restrict__ r, W* __restrict__ p, W* __restrict__ z,
                                                  W* __restrict__ s, W* __restrict__ tv, PcgState* __restrict__ st_p) {
  __shared__ W acc_sh[TB], tmp_sh[TB];
  __shared__ double red[PT / 64];
  __shared__ int s_done;
  PcgState& st = *st_p;
  if (st.outer_done) return;
  for (int64_t i = threadIdx.x; i < m; i += PT) {
    W v = b[i];
    if (parts) {
      W q = parts[i];
      for (int c = 1; c < nparts; ++c) q = vadd(q, parts[(int64_t)c * m + i]);
      v = vsub(v, q);
    }
    r[i] = v;
    y[i] = vzero<W>();
  }
  __syncthreads();
  trsv_adj<RV, W>(R, ldr, X, m, r, s, acc_sh, tmp_sh);
  double rho = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += PT) rho += vabs2(s[i]);
  rho = block_sum(rho, red);
  if (parts) {
    // outer certificate on the FP64 residual: ||x - p|| <= sqrt(rho)/sigma,
    // sigma >= ~0.9 for an R from single-precision data: test against eps/2
    double xi = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += PT) xi += vre(vcmul(y_outer[i], vsub(b[i], r[i])));
    xi = block_sum(xi, red);
    const double e = 0.5 * st.eps_outer;
    const double tol = e / (1.0 + e);
    if (threadIdx.x == 0) {
      st.outer_rho = rho;
      st.outer_xi = xi;
      st.refine_steps += 1;
      if (!(isfinite(rho) && isfinite(xi))) {
        st.outer_done = 1;
        st.status = 4;
      } else if (rho <= tol * tol * xi || (rho == 0.0)) {
        st.outer_done = 1;
      } else if (st.refine_steps > st.max_refine) {
        st.outer_done = 1;
        st.status = 2;
      }
      s_done = st.outer_done;
    }
    __syncthreads();
    if (s_done) {
      if (threadIdx.x == 0) st.done = 1;
      return;
    }
  }
  trsv_fwd<RV, W>(R, ldr, X, m, s, z, tv);
  for (int64_t i = threadIdx.x; i < m; i += PT) p[i] = z[i];
  if (threadIdx.x == 0) {
    st.rho0 = rho;
    st.rho = rho;
    st.xi = 0.0;
    st.iter_local = 0;
    st.done = (rho == 0.0) ? 1 : 0;
    if (!isfinite(rho)) {
      st.done = 1;
      st.status = 4;
    }
  }
}

// One CG iteration's tail, after q = A (A* p) was produced as partial sums.
template <typename RV, typename W>
__global__ void __launch_bounds__(PT) k_pcg_tail(const RV* __restrict__ R, int64_t ldr, const W* __restrict__ X,
                                                 int64_t m, const W* __restrict__ b, const W* __restrict__ qpart,
                                                 int nparts, W* __restrict__ y, W* __restrict__ r, W* __restrict__ p,
                                                 W* __restrict__ z, W* __restrict__ s, W* __restrict__ q,
                                                 W* __restrict__ tv, PcgState* __restrict__ st_p) {
  __shared__ W acc_sh[TB], tmp_sh[TB];
  __shared__ double red[PT / 64];
  __shared__ int s_stop;
  PcgState& st = *st_p;
  if (st.done) return;
  // q = sum of the partial products, and p^* q
  double pq = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += PT) {
    W v = qpart[i];
    for (int c = 1; c < nparts; ++c) v = vadd(v, qpart[(int64_t)c * m + i]);
    q[i] = v;
    pq += vre(vcmul(p[i], v));
  }
  pq = block_sum(pq, red);
  const double rho = st.rho;
  const double alpha = rho / pq;
  const bool bad = !(isfinite(alpha) && pq > 0.0);
  if (bad) {
    if (threadIdx.x == 0) {
      st.done = 1;
      st.status = 4;
    }
    return;
  }
  for (int64_t i = threadIdx.x; i < m; i += PT) {
    y[i] = vadd(y[i], vscale(p[i], alpha));
    r[i] = vsub(r[i], vscale(q[i], alpha));
  }
  __syncthreads();
  trsv_adj<RV, W>(R, ldr, X, m, r, s, acc_sh, tmp_sh);
  double rho_new = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += PT) rho_new += vabs2(s[i]);
  rho_new = block_sum(rho_new, red);
  double xi = 0.0;
  if (st.rule != 2) {
    for (int64_t i = threadIdx.x; i < m; i += PT) xi += vre(vcmul(y[i], vsub(b[i], r[i])));
    xi = block_sum(xi, red);
  }
  if (threadIdx.x == 0) {
    int stop = 0;
    st.iter_local += 1;
    st.iter_total += 1;
    st.rho = rho_new;
    st.xi = xi;
    if (!isfinite(rho_new)) {
      st.status = 4;
      stop = 1;
    } else if (stop_test(st, rho_new, xi)) {
      stop = 1;
    } else if (st.iter_local >= st.max_iter) {
      stop = 1;
      if (st.rule != 2) st.status = 2;
    }
    s_stop = stop;
  }
  __syncthreads();
  if (s_stop) {
    if (threadIdx.x == 0) st.done = 1;
    return;
  }
  trsv_fwd<RV, W>(R, ldr, X, m, s, z, tv);
  const double beta = rho_new / rho;
  for (int64_t i = threadIdx.x; i < m; i += PT) p[i] = vadd(z[i], vscale(p[i], beta));
}

// y_outer += y (after an inner solve); re-arms the inner loop's flag.
template <typename W>
__global__ void k_refine_update(W* __restrict__ y_outer, const W* __restrict__ y, int64_t m, PcgState* st) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (st->outer_done) return;
  if (i < m) y_outer[i] = vadd(y_outer[i], y[i]);
}

template <typename W> __global__ void k_copy_vec(const W* __restrict__ a, W* __restrict__ b, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) b[i] = a[i];
}

// ------------------------------ launchers -----------------------------------
template <typename RV, typename W>
static hipError_t inv_diag_impl(const void* R, int64_t ldr, int64_t m, void* X, hipStream_t st) {
  hipLaunchKernelGGL((k_inv_diag<RV, W>), dim3((unsigned)ceil_div(m, TB)), dim3(256), 0, st,
                     reinterpret_cast<const RV*>(R), ldr, m, reinterpret_cast<W*>(X));
  return hipGetLastError();
}

hipError_t launch_inv_diag(int rdtype, const void* R, int64_t ldr, int64_t m, void* X, hipStream_t st) {
  switch (rdtype) {
    case 0: return inv_diag_impl<cd, cd>(R, ldr, m, X, st);
    case 1: return inv_diag_impl<cf, cd>(R, ldr, m, X, st);
    case 2: return inv_diag_impl<double, double>(R, ldr, m, X, st);
    case 3: return inv_diag_impl<float, double>(R, ldr, m, X, st);
  }
  return hipErrorInvalidValue;
}

template <typename RV, typename W>
static hipError_t start_impl(const PcgVecs& v, const void* parts, int nparts, const void* y_outer, hipStream_t st) {
  hipLaunchKernelGGL((k_pcg_start<RV, W>), dim3(1), dim3(PT), 0, st, reinterpret_cast<const RV*>(v.R), v.ldr,
                     reinterpret_cast<const W*>(v.X), v.m, reinterpret_cast<const W*>(v.b),
                     reinterpret_cast<const W*>(parts), nparts, reinterpret_cast<const W*>(y_outer),
                     reinterpret_cast<W*>(v.y), reinterpret_cast<W*>(v.r), reinterpret_cast<W*>(v.p),
                     reinterpret_cast<W*>(v.z), reinterpret_cast<W*>(v.s), reinterpret_cast<W*>(v.tv), v.state);
  return hipGetLastError();
}

template <typename RV, typename W>
static hipError_t tail_impl(const PcgVecs& v, const void* qpart, int nparts, hipStream_t st) {
  hipLaunchKernelGGL((k_pcg_tail<RV, W>), dim3(1), dim3(PT), 0, st, reinterpret_cast<const RV*>(v.R), v.ldr,
                     reinterpret_cast<const W*>(v.X), v.m, reinterpret_cast<const W*>(v.b),
                     reinterpret_cast<const W*>(qpart), nparts, reinterpret_cast<W*>(v.y),
                     reinterpret_cast<W*>(v.r), reinterpret_cast<W*>(v.p), reinterpret_cast<W*>(v.z),
                     reinterpret_cast<W*>(v.s), reinterpret_cast<W*>(v.q), reinterpret_cast<W*>(v.tv), v.state);
  return hipGetLastError();
}

hipError_t launch_pcg_start(int rdtype, const PcgVecs& v, const void* parts, int nparts, const void* y_outer,
                            hipStream_t st) {
  switch (rdtype) {
    case 0: return start_impl<cd, cd>(v, parts, nparts, y_outer, st);
    case 1: return start_impl<cf, cd>(v, parts, nparts, y_outer, st);
    case 2: return start_impl<double, double>(v, parts, nparts, y_outer, st);
    case 3: return start_impl<float, double>(v, parts, nparts, y_outer, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pcg_tail(int rdtype, const PcgVecs& v, const void* qpart, int nparts, hipStream_t st) {
  switch (rdtype) {
    case 0: return tail_impl<cd, cd>(v, qpart, nparts, st);
    case 1: return tail_impl<cf, cd>(v, qpart, nparts, st);
    case 2: return tail_impl<double, double>(v, qpart, nparts, st);
    case 3: return tail_impl<float, double>(v, qpart, nparts, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_refine_update(bool cplx, void* y_outer, const void* y, int64_t m, PcgState* state,
                                hipStream_t st) {
  if (cplx)
    hipLaunchKernelGGL(k_refine_update<cd>, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st,
                       reinterpret_cast<cd*>(y_outer), reinterpret_cast<const cd*>(y), m, state);
  else
    hipLaunchKernelGGL(k_refine_update<double>, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st,
                       reinterpret_cast<double*>(y_outer), reinterpret_cast<const double*>(y), m, state);
  return hipGetLastError();
}

}  // namespace mn
