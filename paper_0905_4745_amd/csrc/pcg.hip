// Step 4 of the method read as preconditioned conjugate gradients on
// A A* y = b (A c = b by Lemma 5.1 makes these the normal equations of
// eq. overdet), preconditioned by R* R with R from Step 2's factorisation.
//
// The m-vectors of the iteration (y, r, p, z, s, q) are FP64 whatever the
// precision of A; their inner products and norms, and the stopping test,
// are FP64 too.
//
// Preconditioner.  The two triangular solves s = R^{-*} r and z = R^{-1} s are
// applied through X = R^{-1}, formed once per factorisation by blocked
// back substitution on 32 x 32 blocks (diagonal blocks inverted directly, then
// X_ij = -X_ii sum_{i<k<=j} R_ik X_kj one block diagonal at a time), in FP64
// from R promoted out of its storage precision.  Each solve is then one
// triangular matrix-vector product spread over many workgroups, with X (at
// most m^2 / 2 FP64 entries) resident in the last-level cache.
//
// One CG iteration after q = A (A* p) = sum of partial products:
//   k_cg_s  (column blocks of X)  alpha = rho / p^* q; r' = r - alpha q;
//                                 y += alpha p; s = X^* r'
//   k_cg_p  (row bands of X)      rho' = ||s||^2; xi = Re(y^*(b - r'));
//                                 stopping test; z = X s; p = z + (rho'/rho) p
// Scalars every workgroup needs (alpha, rho', xi) are recomputed by each
// workgroup in the same fixed order, so all take identical decisions; only
// workgroup 0 writes the shared vectors y, r' and the state.
//
// Stopping rules, with rho = ||R^{-*} r||^2 and xi = ||A* y||^2
// (||x - p||^2 <= rho since the SRFT has orthonormal rows):
//   rule 0 -- the paper's precision for Step 4, f - f* <= delta f*,
//             delta = eps^2 l / (alpha N): rho <= delta (rho0 - (sqrt xi + sqrt rho)^2)
//             (rule 1 when l = N: then f* = 0);
//   rule 1 -- ||x - p|| <= eps ||p||:  rho <= (eps / (1 + eps))^2 xi;
//   rule 2 -- relative reduction of an inner solve: rho <= eps^2 rho0.
#include "common.hpp"
#include "kernels.hpp"
#include "batch_dev.hpp"

namespace mn {

constexpr int TB = 32;  // block edge of X

// R entry (gi, gk) promoted to FP64, with R extended by the identity beyond m
template <typename RV, typename W>
__device__ inline W r_at(const RV* R, int64_t ldr, int64_t m, int64_t gi, int64_t gk) {
  if (gi < m && gk < m) return vconv<W>(R[gi + gk * ldr]);
  return gi == gk ? vmake<W>(1.0, 0.0) : vzero<W>();
}

// Diagonal blocks X_ii = R_ii^{-1} (back substitution, one thread per
// column of the block).  grid = K blocks, 256 threads.
template <typename RV, typename W>
__device__ __forceinline__ void k_inv_diag_body(const Bk bk, const RV* __restrict__ R, int64_t ldr, int64_t m,
                                                  W* __restrict__ X, int64_t ldx) {
  __shared__ W T[TB * TB];
  __shared__ W Xs[TB * TB];
  const int64_t c0 = (int64_t)bk.x * TB;
  for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) {
    const int r = e % TB, c = e / TB;
    T[e] = r_at<RV, W>(R, ldr, m, c0 + r, c0 + c);
    Xs[e] = vzero<W>();
  }
  __syncthreads();
  if (threadIdx.x < TB) {
    const int c = threadIdx.x;
    for (int i = c; i >= 0; --i) {
      W acc = (i == c) ? vmake<W>(1.0, 0.0) : vzero<W>();
      for (int j = i + 1; j <= c; ++j) acc = vsub(acc, vmul(T[i + j * TB], Xs[j + c * TB]));
      const W d = T[i + i * TB];
      Xs[i + c * TB] = vscale(vcmul(d, acc), 1.0 / vabs2(d));  // acc / d
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) {
    const int r = e % TB, c = e / TB;
    X[(c0 + r) + (c0 + c) * ldx] = Xs[e];
  }
}
template <typename RV, typename W>
__global__ void __launch_bounds__(256) k_inv_diag(const RV* __restrict__ R, int64_t ldr, int64_t m,
                                                  W* __restrict__ X, int64_t ldx) {
  k_inv_diag_body<RV, W>(bk_hw(), R, ldr, m, X, ldx);
}

// Off-diagonal blocks, right-looking: in block step k (block column k of X
// final: X_ik for i <= k) every tile (i, j), i <= k < j, adds X_ik R_kj to the
// running sum held in X_ij (stored, not added, for its first term k = i); the
// tiles of column j = k + 1 then hold the whole sum S and are finished as
// X_{i,k+1} = -S X_{k+1,k+1}.  Each workgroup does one or two 32 x 32
// products, so the chain is K - 1 short launches.  grid = (k + 1)(K - k - 1).
constexpr int LDT = TB + 1;  // LDS column stride

// acc[u] += A(r, q) B(q, cg + 8u); thread t: row r = t % 32, columns cg + 8u
template <typename W>
__device__ __forceinline__ void tile_mm32(const W* A, const W* B, W acc[4]) {
  const int r = threadIdx.x % TB, cg = threadIdx.x / TB;
#pragma unroll 8
  for (int q = 0; q < TB; ++q) {
    const W a = A[r + q * LDT];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = vfma(a, B[q + (cg + 8 * u) * LDT], acc[u]);
  }
}

template <typename RV, typename W>
__device__ __forceinline__ void k_trtri_step_body(const Bk bk, const RV* __restrict__ R, int64_t ldr, int64_t m,
                                                    W* __restrict__ X, int64_t ldx, int k, int K) {
  __shared__ W As[TB * LDT];
  __shared__ W Bs[TB * LDT];
  const int ncol = K - k - 1;
  const int i = bk.x / ncol, j = k + 1 + bk.x % ncol;
  const int64_t i0 = (int64_t)i * TB, j0 = (int64_t)j * TB, k0 = (int64_t)k * TB;
  const int r = threadIdx.x % TB, cg = threadIdx.x / TB;
  W acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = cg + 8 * u;
    As[r + c * LDT] = X[(i0 + r) + (k0 + c) * ldx];         // X_ik
    Bs[r + c * LDT] = r_at<RV, W>(R, ldr, m, k0 + r, j0 + c);  // R_kj
    acc[u] = (k == i) ? vzero<W>() : X[(i0 + r) + (j0 + c) * ldx];
  }
  __syncthreads();
  tile_mm32(As, Bs, acc);
  if (j == k + 1) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = cg + 8 * u;
      As[r + c * LDT] = acc[u];                             // S
      Bs[r + c * LDT] = X[(j0 + r) + (j0 + c) * ldx];       // X_jj
    }
    __syncthreads();
    W o[4] = {vzero<W>(), vzero<W>(), vzero<W>(), vzero<W>()};
    tile_mm32(As, Bs, o);
#pragma unroll
    for (int u = 0; u < 4; ++u) X[(i0 + r) + (j0 + cg + 8 * u) * ldx] = vsub(vzero<W>(), o[u]);
    return;
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) X[(i0 + r) + (j0 + cg + 8 * u) * ldx] = acc[u];
}
template <typename RV, typename W>
__global__ void __launch_bounds__(256) k_trtri_step(const RV* __restrict__ R, int64_t ldr, int64_t m,
                                                    W* __restrict__ X, int64_t ldx, int k, int K) {
  k_trtri_step_body<RV, W>(bk_hw(), R, ldr, m, X, ldx, k, K);
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

// ---------------------------------------------------------------------------
// k_cg_s.  start: r' = b - sum(parts) (or b), y = 0.  iter: alpha, r', y.
// Then s_j = sum_{i<=j} conj(X_ij) r'_i for this workgroup's 4 CPW columns
// (CPW = 2, or 1 for large m, where the longer columns want more waves in
// flight).  grid = ceil(m / (4 CPW)), 256 threads, dynamic LDS = m FP64
// entries (r').
template <typename W, int CPW = 2>
__device__ __forceinline__ void k_cg_s_body(const Bk bk, const W* __restrict__ X, int64_t ldx, int64_t m, int start,
                                              const W* __restrict__ b, const W* __restrict__ parts, int nparts,
                                              W* __restrict__ p, W* __restrict__ y, const W* __restrict__ r_in,
                                              W* __restrict__ r_out, W* __restrict__ s, PcgState* __restrict__ stp) {
  extern __shared__ unsigned char smem_raw[];
  W* rs = reinterpret_cast<W*>(smem_raw);
  __shared__ double red[4];
  PcgState& st = *stp;
  const bool lead = bk.x == 0;
  // s for this workgroup's columns: wave w takes CPW of them, lanes run down
  // each.  Column j of X has entries 0 .. j; its first 256 entries do not
  // depend on the iteration, so their loads are issued before anything else.
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t j0 = (int64_t)bk.x * (4 * CPW) + CPW * wv, j1 = j0 + 1;
  const int64_t e0 = j0 < m ? j0 + 1 : 0, e1 = (CPW == 2 && j1 < m) ? j1 + 1 : 0;
  const W* col0 = X + j0 * ldx;
  const W* col1 = X + j1 * ldx;
  W x0[4], x1[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t ii = lane + 64 * u;
    x0[u] = ii < e0 ? col0[ii] : vzero<W>();
    x1[u] = ii < e1 ? col1[ii] : vzero<W>();
  }
  if (start) {
    if (st.outer_done) return;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
      W v = b[i];
      if (parts) {
        W q = parts[i];
        for (int c = 1; c < nparts; ++c) q = vadd(q, parts[(int64_t)c * m + i]);
        v = vsub(v, q);
      }
      rs[i] = v;
      if (lead) {
        r_out[i] = v;
        y[i] = vzero<W>();
      }
    }
    if (lead && threadIdx.x == 0) st.refine_snap = st.refine_steps + (parts ? 1 : 0);
  } else {
    if (st.done) return;
    // q = sum of the partial products (kept in p-order), alpha = rho / p^* q.
    // For the first 1024 entries the iteration's other vectors (r, and p, y
    // in the lead workgroup) are loaded together with q's slices.
    constexpr int PF = 4;
    double pq = 0.0;
    W rv[PF], pv[PF], yv[PF];
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int64_t i = threadIdx.x + 256 * t;
      rv[t] = pv[t] = yv[t] = vzero<W>();
      if (i < m) {
        W q = parts[i];
        for (int c = 1; c < nparts; ++c) q = vadd(q, parts[(int64_t)c * m + i]);
        pv[t] = p[i];
        rv[t] = r_in[i];
        if (lead) yv[t] = y[i];
        rs[i] = q;
        pq += vre(vcmul(pv[t], q));
      }
    }
    for (int64_t i = threadIdx.x + 256 * PF; i < m; i += blockDim.x) {
      W q = parts[i];
      for (int c = 1; c < nparts; ++c) q = vadd(q, parts[(int64_t)c * m + i]);
      rs[i] = q;
      pq += vre(vcmul(p[i], q));
    }
    pq = block_sum(pq, red);
    const double alpha = st.rho / pq;
    if (!(isfinite(alpha) && pq > 0.0)) {
      if (lead && threadIdx.x == 0) {
        st.done = 1;
        st.status = 4;
      }
      return;
    }
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int64_t i = threadIdx.x + 256 * t;
      if (i < m) {
        const W v = vsub(rv[t], vscale(rs[i], alpha));
        rs[i] = v;
        if (lead) {
          r_out[i] = v;
          y[i] = vadd(yv[t], vscale(pv[t], alpha));
        }
      }
    }
    for (int64_t i = threadIdx.x + 256 * PF; i < m; i += blockDim.x) {
      const W v = vsub(r_in[i], vscale(rs[i], alpha));
      rs[i] = v;
      if (lead) {
        r_out[i] = v;
        y[i] = vadd(y[i], vscale(p[i], alpha));
      }
    }
    if (lead && threadIdx.x == 0) {
      st.rho_prev = st.rho;
      st.iter_snap = st.iter_local;
    }
  }
  __syncthreads();
  // both columns are walked together with four accumulators each, so all of
  // a lane's loads are in flight at once
  W a0[4] = {vzero<W>(), vzero<W>(), vzero<W>(), vzero<W>()};
  W a1[4] = {vzero<W>(), vzero<W>(), vzero<W>(), vzero<W>()};
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t ii = lane + 64 * u;
    if (ii < e0) a0[u] = vcfma(x0[u], rs[ii], a0[u]);
    if (ii < e1) a1[u] = vcfma(x1[u], rs[ii], a1[u]);
  }
  const int64_t emax = e0 > e1 ? e0 : e1;
  for (int64_t i = lane + 256; i < emax; i += 256) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t ii = i + 64 * u;
      if (ii < e0) a0[u] = vcfma(col0[ii], rs[ii], a0[u]);
      if (ii < e1) a1[u] = vcfma(col1[ii], rs[ii], a1[u]);
    }
  }
  W acc0 = wave_sum(vadd(vadd(a0[0], a0[1]), vadd(a0[2], a0[3])));
  W acc1 = wave_sum(vadd(vadd(a1[0], a1[1]), vadd(a1[2], a1[3])));
  if (lane == 0) {
    if (j0 < m) s[j0] = acc0;
    if (CPW == 2 && j1 < m) s[j1] = acc1;
  }
}
template <typename W, int CPW = 2>
__global__ void __launch_bounds__(256) k_cg_s(const W* __restrict__ X, int64_t ldx, int64_t m, int start,
                                              const W* __restrict__ b, const W* __restrict__ parts, int nparts,
                                              W* __restrict__ p, W* __restrict__ y, const W* __restrict__ r_in,
                                              W* __restrict__ r_out, W* __restrict__ s, PcgState* __restrict__ stp) {
  k_cg_s_body<W, CPW>(bk_hw(), X, ldx, m, start, b, parts, nparts, p, y, r_in, r_out, s, stp);
}

// ---------------------------------------------------------------------------
// k_cg_p.  rho' = ||s||^2 (and xi, the stopping test); z = X s on this
// workgroup's RB-row band; p = z + beta p (start: p = z, rho0 = rho').
// With y_outer (start of an FP64 refinement step) the outer certificate is
// tested first.  grid = ceil(m / RB), 256 threads (RB = 16, or 8 for large
// m, where 16-row bands leave half the CUs without a workgroup).
template <typename W, int RB = 16>
__device__ __forceinline__ void k_cg_p_body(const Bk bk, const W* __restrict__ X, int64_t ldx, int64_t m, int start,
                                              const W* __restrict__ b, const W* __restrict__ y,
                                              const W* __restrict__ y_outer, const W* __restrict__ r,
                                              const W* __restrict__ s, W* __restrict__ p,
                                              PcgState* __restrict__ stp) {
  constexpr int NG = 256 / RB;  // column groups
  extern __shared__ unsigned char smem_raw[];
  W* ss = reinterpret_cast<W*>(smem_raw);  // s, m entries
  __shared__ W part[NG][RB];
  PcgState& st = *stp;
  const bool lead = bk.x == 0;
  // z = X s on rows i0 .. i0+RB-1: thread t takes row t%RB and every NG-th
  // column.  X is zero below the diagonal inside the diagonal block, so the
  // band can be read from column i0 on; the first group of four columns per
  // thread does not depend on the iteration and is loaded first.
  const int64_t i0 = (int64_t)bk.x * RB;
  const int rr = threadIdx.x % RB, cgrp = threadIdx.x / RB;
  const int64_t i = i0 + rr;
  const bool first = i < m && i0 + cgrp + 3 * NG < m;
  W xf[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) xf[u] = first ? X[i + (i0 + cgrp + NG * u) * ldx] : vzero<W>();
  const int64_t ip = i0 + threadIdx.x;  // this workgroup's entries of p (threads < 16)
  const W p_old = (!start && threadIdx.x < RB && ip < m) ? p[ip] : vzero<W>();
  if (start ? (st.outer_done != 0) : (st.done != 0)) return;
  // rho = ||s||^2 and, where the stopping test needs it, xi = Re(y* (b - r))
  // (y_outer at the start of a refinement step): one pass, one reduction
  const W* yx = start ? y_outer : y;
  const bool want_xi = start ? (y_outer != nullptr) : (st.rule != 2);
  cd rx = cd{0.0, 0.0};
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
    const W v = s[i];
    ss[i] = v;
    rx.re += vabs2(v);
    if (want_xi) rx.im += vre(vcmul(yx[i], vsub(b[i], r[i])));
  }
  __shared__ cd redc[4];
  rx = block_sum(rx, redc);
  const double rho = rx.re;
  double beta = 0.0;
  if (start) {
    if (y_outer) {
      // FP64 certificate of the current outer iterate: ||x - p|| <= sqrt(rho)/sigma
      // with sigma >= ~0.9 for an R from single-precision data: test eps/2
      const double xi = rx.im;
      const double e = 0.5 * st.eps_outer;
      const double tol = e / (1.0 + e);
      int od = 0, status = st.status;
      if (!(isfinite(rho) && isfinite(xi))) {
        od = 1;
        status = 4;
      } else if (rho <= tol * tol * xi || rho == 0.0) {
        od = 1;
      } else if (st.refine_snap > st.max_refine) {
        od = 1;
        status = 2;
      }
      if (lead && threadIdx.x == 0) {
        st.outer_rho = rho;
        st.outer_xi = xi;
        st.refine_steps = st.refine_snap;
        st.status = status;
        if (od) {
          st.outer_done = 1;
          st.done = 1;
        }
      }
      if (od) return;
    }
    if (lead && threadIdx.x == 0) {
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
    if (rho == 0.0 || !isfinite(rho)) return;
  } else {
    const double xi = want_xi ? rx.im : 0.0;
    const int it = st.iter_snap + 1;
    int stop = 0, status = st.status;
    if (!isfinite(rho)) {
      stop = 1;
      status = 4;
    } else if (stop_test(st, rho, xi)) {
      stop = 1;
    } else if (it >= st.max_iter) {
      stop = 1;
      if (st.rule != 2) status = 2;
    }
    if (lead && threadIdx.x == 0) {
      st.iter_local = it;
      st.iter_total += 1;
      st.rho = rho;
      st.xi = xi;
      st.status = status;
      if (stop) st.done = 1;
    }
    if (stop) return;
    beta = rho / st.rho_prev;
  }
  // four independent accumulators keep the loads of a thread in flight
  // together
  W a4[4] = {vzero<W>(), vzero<W>(), vzero<W>(), vzero<W>()};
  if (i < m) {
    int64_t j = i0 + cgrp;
    if (first) {
#pragma unroll
      for (int u = 0; u < 4; ++u) a4[u] = vfma(xf[u], ss[j + NG * u], a4[u]);
      j += 4 * NG;
    }
    for (; j + 3 * NG < m; j += 4 * NG) {
#pragma unroll
      for (int u = 0; u < 4; ++u) a4[u] = vfma(X[i + (j + NG * u) * ldx], ss[j + NG * u], a4[u]);
    }
    for (; j < m; j += NG) a4[0] = vfma(X[i + j * ldx], ss[j], a4[0]);
  }
  W acc = vadd(vadd(a4[0], a4[1]), vadd(a4[2], a4[3]));
  part[cgrp][rr] = acc;
  __syncthreads();
  if (threadIdx.x < RB && i0 + threadIdx.x < m) {
    W z = part[0][threadIdx.x];
    for (int c = 1; c < NG; ++c) z = vadd(z, part[c][threadIdx.x]);
    const int64_t ii = i0 + threadIdx.x;
    p[ii] = start ? z : vadd(z, vscale(p_old, beta));
  }
}
template <typename W, int RB = 16>
__global__ void __launch_bounds__(256) k_cg_p(const W* __restrict__ X, int64_t ldx, int64_t m, int start,
                                              const W* __restrict__ b, const W* __restrict__ y,
                                              const W* __restrict__ y_outer, const W* __restrict__ r,
                                              const W* __restrict__ s, W* __restrict__ p,
                                              PcgState* __restrict__ stp) {
  k_cg_p_body<W, RB>(bk_hw(), X, ldx, m, start, b, y, y_outer, r, s, p, stp);
}

// y_outer += y (after an inner solve).
template <typename W>
__device__ __forceinline__ void k_refine_update_body(const Bk bk, W* __restrict__ y_outer, const W* __restrict__ y, int64_t m, const PcgState* st) {
  const int64_t i = (int64_t)bk.x * blockDim.x + threadIdx.x;
  if (st->outer_done) return;
  if (i < m) y_outer[i] = vadd(y_outer[i], y[i]);
}
template <typename W>
__global__ void k_refine_update(W* __restrict__ y_outer, const W* __restrict__ y, int64_t m, const PcgState* st) {
  k_refine_update_body<W>(bk_hw(), y_outer, y, m, st);
}

template <typename W> __device__ __forceinline__ void k_zero_vec_body(const Bk bk, W* __restrict__ v, int64_t m) {
  const int64_t i = (int64_t)bk.x * blockDim.x + threadIdx.x;
  if (i < m) v[i] = vzero<W>();
}
template <typename W> __global__ void k_zero_vec(W* __restrict__ v, int64_t m) {
  k_zero_vec_body<W>(bk_hw(), v, m);
}

// ------------------------------ launchers -----------------------------------
template <typename RV, typename W>
static hipError_t inverse_impl(const void* R, int64_t ldr, int64_t m, void* X, int64_t ldx, hipStream_t st) {
  const int K = (int)ceil_div(m, TB);
  hipLaunchKernelGGL((k_inv_diag<RV, W>), dim3(K), dim3(256), 0, st, reinterpret_cast<const RV*>(R), ldr, m,
                     reinterpret_cast<W*>(X), ldx);
  for (int k = 0; k + 1 < K; ++k)
    hipLaunchKernelGGL((k_trtri_step<RV, W>), dim3((k + 1) * (K - k - 1)), dim3(256), 0, st,
                       reinterpret_cast<const RV*>(R), ldr, m, reinterpret_cast<W*>(X), ldx, k, K);
  return hipGetLastError();
}

int64_t rinv_ld(int64_t m) { return ceil_div(m, TB) * TB; }

hipError_t launch_rinv(int rdtype, const void* R, int64_t ldr, int64_t m, void* X, hipStream_t st) {
  const int64_t ldx = rinv_ld(m);
  switch (rdtype) {
    case 0: return inverse_impl<cd, cd>(R, ldr, m, X, ldx, st);
    case 1: return inverse_impl<cf, cd>(R, ldr, m, X, ldx, st);
    case 2: return inverse_impl<double, double>(R, ldr, m, X, ldx, st);
    case 3: return inverse_impl<float, double>(R, ldr, m, X, ldx, st);
  }
  return hipErrorInvalidValue;
}

template <typename W>
static hipError_t cg_step_impl(const CgStep& a, hipStream_t st) {
  const W* X = reinterpret_cast<const W*>(a.X);
  const int64_t ldx = rinv_ld(a.m);
  const size_t sm = (size_t)a.m * sizeof(W);
  if (sm > 48 * 1024) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_cg_s<W>), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sm);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_cg_s<W, 1>), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sm);
  }
  if (sm > 48 * 1024) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_cg_p<W>), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sm);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_cg_p<W, 8>), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sm);
  }
  if (a.m >= 1024)
    hipLaunchKernelGGL((k_cg_s<W, 1>), dim3((unsigned)ceil_div(a.m, 4)), dim3(256), sm, st, X, ldx, a.m, a.start,
                       reinterpret_cast<const W*>(a.b), reinterpret_cast<const W*>(a.parts), a.nparts,
                       reinterpret_cast<W*>(a.p), reinterpret_cast<W*>(a.y), reinterpret_cast<const W*>(a.r_in),
                       reinterpret_cast<W*>(a.r_out), reinterpret_cast<W*>(a.s), a.state);
  else
    hipLaunchKernelGGL((k_cg_s<W>), dim3((unsigned)ceil_div(a.m, 8)), dim3(256), sm, st, X, ldx, a.m, a.start,
                       reinterpret_cast<const W*>(a.b), reinterpret_cast<const W*>(a.parts), a.nparts,
                       reinterpret_cast<W*>(a.p), reinterpret_cast<W*>(a.y), reinterpret_cast<const W*>(a.r_in),
                       reinterpret_cast<W*>(a.r_out), reinterpret_cast<W*>(a.s), a.state);
  if (a.m >= 1024)
    hipLaunchKernelGGL((k_cg_p<W, 8>), dim3((unsigned)ceil_div(a.m, 8)), dim3(256), sm, st, X, ldx, a.m, a.start,
                       reinterpret_cast<const W*>(a.b), reinterpret_cast<const W*>(a.y),
                       reinterpret_cast<const W*>(a.y_outer), reinterpret_cast<const W*>(a.r_out),
                       reinterpret_cast<const W*>(a.s), reinterpret_cast<W*>(a.p), a.state);
  else
    hipLaunchKernelGGL((k_cg_p<W>), dim3((unsigned)ceil_div(a.m, 16)), dim3(256), sm, st, X, ldx, a.m, a.start,
                       reinterpret_cast<const W*>(a.b), reinterpret_cast<const W*>(a.y),
                       reinterpret_cast<const W*>(a.y_outer), reinterpret_cast<const W*>(a.r_out),
                       reinterpret_cast<const W*>(a.s), reinterpret_cast<W*>(a.p), a.state);
  return hipGetLastError();
}

hipError_t launch_cg_step(bool cplx, const CgStep& a, hipStream_t st) {
  return cplx ? cg_step_impl<cd>(a, st) : cg_step_impl<double>(a, st);
}

hipError_t launch_refine_update(bool cplx, void* y_outer, const void* y, int64_t m, const PcgState* state,
                                hipStream_t st) {
  if (cplx)
    hipLaunchKernelGGL(k_refine_update<cd>, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st,
                       reinterpret_cast<cd*>(y_outer), reinterpret_cast<const cd*>(y), m, state);
  else
    hipLaunchKernelGGL(k_refine_update<double>, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st,
                       reinterpret_cast<double*>(y_outer), reinterpret_cast<const double*>(y), m, state);
  return hipGetLastError();
}

hipError_t launch_zero(bool cplx, void* v, int64_t m, hipStream_t st) {
  if (cplx)
    hipLaunchKernelGGL(k_zero_vec<cd>, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, reinterpret_cast<cd*>(v),
                       m);
  else
    hipLaunchKernelGGL(k_zero_vec<double>, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st,
                       reinterpret_cast<double*>(v), m);
  return hipGetLastError();
}

// ------------------------------ batched systems -------------------------------
namespace {

template <typename W>
__global__ void __launch_bounds__(256) kb_inv_diag(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                   int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_inv_diag_body<W, W>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<const W*>(s.R), s.m,
                        s.m, reinterpret_cast<W*>(s.X), s.ldx);
}

template <typename W>
__global__ void __launch_bounds__(256) kb_trtri_step(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                     int nsys, int k) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_trtri_step_body<W, W>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<const W*>(s.R),
                          s.m, s.m, reinterpret_cast<W*>(s.X), s.ldx, k, (int)ceil_div(s.m, TB));
}

// r ping-pong: at iteration parity par, r_in = r[par] and r_out = r[par ^ 1];
// a start writes r[par]
template <typename W>
__device__ inline W* r_buf(const BSys& s, int which) {
  return reinterpret_cast<W*>(which ? s.r1 : s.r0);
}

template <typename W>
__global__ void __launch_bounds__(256) kb_cg_s(const BSys* __restrict__ sys, const BGrid* __restrict__ grid, int nsys,
                                               int start, int parts, int par) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  const W* pp = parts == 1 ? reinterpret_cast<const W*>(s.fpart) : parts == 2 ? reinterpret_cast<const W*>(s.q) : nullptr;
  const int np = parts == 1 ? s.fwd_chunks : parts == 2 ? kGramParts : 0;
  k_cg_s_body<W>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<const W*>(s.X), s.ldx, s.m,
                 start, reinterpret_cast<const W*>(s.b), pp, np, reinterpret_cast<W*>(s.p), reinterpret_cast<W*>(s.y),
                 start ? nullptr : r_buf<W>(s, par), start ? r_buf<W>(s, par) : r_buf<W>(s, par ^ 1),
                 reinterpret_cast<W*>(s.s), s.st);
}

template <typename W>
__global__ void __launch_bounds__(256) kb_cg_p(const BSys* __restrict__ sys, const BGrid* __restrict__ grid, int nsys,
                                               int start, int outer, int par) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_cg_p_body<W>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<const W*>(s.X), s.ldx, s.m,
                 start, reinterpret_cast<const W*>(s.b), reinterpret_cast<const W*>(s.y),
                 outer ? reinterpret_cast<const W*>(s.y_outer) : nullptr,
                 start ? r_buf<W>(s, par) : r_buf<W>(s, par ^ 1), reinterpret_cast<const W*>(s.s),
                 reinterpret_cast<W*>(s.p), s.st);
}

template <typename W>
__global__ void __launch_bounds__(256) kb_refine(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                 int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_refine_update_body<W>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<W*>(s.y_outer),
                          reinterpret_cast<const W*>(s.y), s.m, s.st);
}

template <typename W>
__global__ void __launch_bounds__(256) kb_zero_outer(const BSys* __restrict__ sys, const BGrid* __restrict__ grid,
                                                     int nsys) {
  const int i = bgrid_find(grid, nsys, blockIdx.x);
  const BSys& s = sys[i];
  k_zero_vec_body<W>(bgrid_local(grid[i], (int)blockIdx.x - grid[i].start), reinterpret_cast<W*>(s.y_outer), s.m);
}

template <typename W>
hipError_t b_cg_t(const BLaunch& Ls, const BLaunch& Lp, int start, int parts, int outer, int par, size_t lds,
                  hipStream_t st) {
  if (lds > 48 * 1024) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kb_cg_s<W>), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kb_cg_p<W>), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  }
  hipLaunchKernelGGL(kb_cg_s<W>, dim3((unsigned)Ls.total), dim3(256), lds, st, Ls.sys, Ls.grid, Ls.nsys, start, parts,
                     par);
  hipLaunchKernelGGL(kb_cg_p<W>, dim3((unsigned)Lp.total), dim3(256), lds, st, Lp.sys, Lp.grid, Lp.nsys, start, outer,
                     par);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_b_inv_diag(bool cplx, const BLaunch& L, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  if (cplx) hipLaunchKernelGGL(kb_inv_diag<cd>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys);
  else hipLaunchKernelGGL(kb_inv_diag<double>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys);
  return hipGetLastError();
}

// block step k of every system with more than k + 1 block columns
hipError_t launch_b_trtri_step(bool cplx, const BLaunch& L, int k, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  if (cplx)
    hipLaunchKernelGGL(kb_trtri_step<cd>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys, k);
  else
    hipLaunchKernelGGL(kb_trtri_step<double>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys, k);
  return hipGetLastError();
}

hipError_t launch_b_cg(bool cplx, const BLaunch& Ls, const BLaunch& Lp, int start, int parts, int outer, int par,
                       size_t lds, hipStream_t st) {
  return cplx ? b_cg_t<cd>(Ls, Lp, start, parts, outer, par, lds, st)
              : b_cg_t<double>(Ls, Lp, start, parts, outer, par, lds, st);
}

hipError_t launch_b_refine(bool cplx, const BLaunch& L, hipStream_t st) {
  if (cplx) hipLaunchKernelGGL(kb_refine<cd>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys);
  else hipLaunchKernelGGL(kb_refine<double>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys);
  return hipGetLastError();
}

hipError_t launch_b_zero_outer(bool cplx, const BLaunch& L, hipStream_t st) {
  if (cplx) hipLaunchKernelGGL(kb_zero_outer<cd>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys);
  else hipLaunchKernelGGL(kb_zero_outer<double>, dim3((unsigned)L.total), dim3(256), 0, st, L.sys, L.grid, L.nsys);
  return hipGetLastError();
}

}  // namespace mn
