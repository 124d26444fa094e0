// The factor H of the SRFT (Section 3, eqs. Rokhlin_trans and big_def):
//   H = Theta Pi Z Theta~ Pi~ Z~,
// Z, Z~ diagonal with unit-modulus entries (+-1 for real data), Pi, Pi~
// permutations ((Pi w)[j] = w[perm[j]]), and Theta = R_1 R_2 ... R_{N-1} a
// chain of plane rotations, R_k acting on coordinates (k-1, k) (zero-based)
// with the block [[c_k, s_k], [-s_k, c_k]], c_k = cos theta_k, s_k = sin theta_k.
// With H, Step 1's transform is T = S F D H, so each row's sketch is
// F(d o H conj(a_i)) at the kept indices; H is applied here to every row and
// the usual sketch kernels transform the result.
//
// Theta w, rightmost rotation first, is a first-order linear recurrence run
// from the last coordinate to the first:
//   t_{N-1} = w[N-1];  t_{k-1} = s_k t_k + c_k w[k-1]        (k = N-1 .. 1)
//   (Theta w)[k] = -s_k w[k-1] + c_k t_k  (k >= 1),   (Theta w)[0] = t_0.
// Writing t_k = s_{k+1} t_{k+1} + c_{k+1} w[k] with (c_N, s_N) = (1, 0), each
// step is an affine map t -> a t + b, so a row is a suffix scan of affine maps:
// one workgroup per row takes chunks of 4096 coordinates from the right; a
// thread composes the maps of its 16 coordinates, the workgroup scans the 256
// composites (Hillis-Steele through LDS, the carry from the chunk to the
// right applied last) and each thread replays its coordinates with the
// carry it receives.  The gather w[k] = zeta[perm[k]] v[perm[k]] (Pi Z v)
// comes first in the same pass, from the source row in global memory.
#include "common.hpp"
#include "kernels.hpp"

namespace mn {

// (c_k, s_k) of R_k for k = 1 .. N-1 at cs[k] (cs[0] unused), in FP64
__global__ void __launch_bounds__(256) k_h_rotations(const double* __restrict__ theta, int64_t N,
                                                     double2* __restrict__ cs) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < 1 || k >= N) return;
  double s, c;
  sincos(theta[k - 1], &s, &c);
  cs[k] = double2{c, s};
}

// out = ProdPi_Z: one stage "Theta Pi Z" of H on rows of src (row r at src +
// r ld_src, entries at or beyond n_src are zero), conj(src) first when
// CONJ_IN, conj(result) stored when CONJ_OUT.  grid = rows, 256 threads.
template <typename V, typename C, bool CONJ_IN, bool CONJ_OUT>
__global__ void __launch_bounds__(256) k_h_stage(const V* __restrict__ src, int64_t ld_src, int64_t n_src,
                                                 V* __restrict__ dst, int64_t ld_dst, int64_t N,
                                                 const int32_t* __restrict__ perm, const void* __restrict__ zeta,
                                                 const double2* __restrict__ cs) {
  constexpr int E = 16, T = 256, CH = E * T;
  using R = typename VT<C>::real;
  __shared__ R sa[2][T];
  __shared__ C sb[2][T];
  const int tid = threadIdx.x;
  const V* row = src + (int64_t)blockIdx.x * ld_src;
  V* out = dst + (int64_t)blockIdx.x * ld_dst;
  auto gather = [&](int64_t k) -> C {
    const uint32_t p = (uint32_t)perm[k];
    if ((int64_t)p >= N) return vzero<C>();  // out-of-range entries (flagged on the host side) read as zero
    C v = (int64_t)p < n_src ? vconv<C>(row[p]) : vzero<C>();
    if constexpr (CONJ_IN) v = vconj(v);
    if constexpr (VT<C>::cplx) {
      const cd z = reinterpret_cast<const cd*>(zeta)[p];
      return vmul(v, vmake<C>(z.re, z.im));
    } else {
      return vscale(v, (R) reinterpret_cast<const double*>(zeta)[p]);
    }
  };
  auto rot = [&](int64_t k) -> double2 { return k < N ? cs[k] : double2{1.0, 0.0}; };
  C carry = vzero<C>();  // t at the right end of the current chunk (t_N = 0)
  for (int64_t hi = N; hi > 0; hi -= CH) {
    const int64_t lo = hi > CH ? hi - CH : 0;
    const int64_t j0 = lo + (int64_t)tid * E;
    const int64_t j1 = (j0 + E) < hi ? (j0 + E) : hi;
    // w[j0 - 1 .. j1 - 1]: the thread's coordinates and its left neighbour
    C w[E + 1];
#pragma unroll
    for (int e = 0; e <= E; ++e) {
      const int64_t k = j0 - 1 + e;
      w[e] = (k >= 0 && k < j1) ? gather(k) : vzero<C>();
    }
    // composite of the thread's maps t_k = s_{k+1} t_{k+1} + c_{k+1} w[k],
    // k = j1 - 1 .. j0:  t_{j0} = a t_{j1} + b
    R a = (R)1;
    C b = vzero<C>();
#pragma unroll
    for (int e = E - 1; e >= 0; --e) {
      const int64_t k = j0 + e;
      if (k < j1) {
        const double2 r = rot(k + 1);
        a = (R)r.y * a;
        b = vadd(vscale(b, (R)r.y), vscale(w[e + 1], (R)r.x));
      }
    }
    // suffix scan over the threads: after it, (a, b) maps t at the chunk's
    // right end to t_{j0} (threads to the right composed first)
    int buf = 0;
    sa[buf][tid] = a;
    sb[buf][tid] = b;
    __syncthreads();
    for (int d = 1; d < T; d <<= 1) {
      R na = sa[buf][tid];
      C nb = sb[buf][tid];
      if (tid + d < T) {
        const R ra = sa[buf][tid + d];
        const C rb = sb[buf][tid + d];
        nb = vadd(vscale(rb, na), nb);  // own map applied after the right one
        na = na * ra;
      }
      sa[buf ^ 1][tid] = na;
      sb[buf ^ 1][tid] = nb;
      buf ^= 1;
      __syncthreads();
    }
    // t_{j1} from the exclusive suffix (the next thread's inclusive one)
    C t = carry;
    if (tid + 1 < T) t = vadd(vscale(carry, sa[buf][tid + 1]), sb[buf][tid + 1]);
    const C next_carry = vadd(vscale(carry, sa[buf][0]), sb[buf][0]);  // t_lo
    // replay: t_k and the outputs of the thread's coordinates
#pragma unroll
    for (int e = E - 1; e >= 0; --e) {
      const int64_t k = j0 + e;
      if (k < j1) {
        const double2 r1 = rot(k + 1);
        t = vadd(vscale(t, (R)r1.y), vscale(w[e + 1], (R)r1.x));
        C o = t;
        if (k >= 1) {
          const double2 r = rot(k);
          o = vsub(vscale(t, (R)r.x), vscale(w[e], (R)r.y));
        }
        if constexpr (CONJ_OUT) o = vconj(o);
        out[k] = vconv<V>(o);
      }
    }
    carry = next_carry;
    __syncthreads();  // the scan buffers are reused by the next chunk
  }
}

// flags perm entries outside [0, N) in *bad (bad must start at zero)
__global__ void __launch_bounds__(256) k_h_check_perm(const int32_t* __restrict__ perm, int64_t N,
                                                      int32_t* __restrict__ bad) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < N && (perm[k] < 0 || (int64_t)perm[k] >= N)) atomicOr(bad, 1);
}

hipError_t launch_h_rotations(const double* theta, int64_t N, double* cs, hipStream_t st) {
  hipLaunchKernelGGL(k_h_rotations, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, st, theta, N,
                     reinterpret_cast<double2*>(cs));
  return hipGetLastError();
}

hipError_t launch_h_check_perm(const int32_t* perm, int64_t N, int32_t* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_h_check_perm, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, st, perm, N, bad);
  return hipGetLastError();
}

template <typename V, typename C>
static hipError_t h_rows_t(bool first, const void* src, int64_t ld_src, int64_t n_src, void* dst, int64_t ld_dst,
                           int64_t rows, int64_t N, const int32_t* perm, const void* zeta, const double* cs,
                           hipStream_t st) {
  const V* s = reinterpret_cast<const V*>(src);
  V* d = reinterpret_cast<V*>(dst);
  const double2* c2 = reinterpret_cast<const double2*>(cs);
  constexpr bool CP = VT<C>::cplx;
  if (first)
    hipLaunchKernelGGL((k_h_stage<V, C, CP, false>), dim3((unsigned)rows), dim3(256), 0, st, s, ld_src, n_src, d,
                       ld_dst, N, perm, zeta, c2);
  else
    hipLaunchKernelGGL((k_h_stage<V, C, false, CP>), dim3((unsigned)rows), dim3(256), 0, st, s, ld_src, n_src, d,
                       ld_dst, N, perm, zeta, c2);
  return hipGetLastError();
}

hipError_t launch_h_rows(int dtype, bool first, const void* src, int64_t ld_src, int64_t n_src, void* dst,
                         int64_t ld_dst, int64_t rows, int64_t N, const int32_t* perm, const void* zeta,
                         const double* cs, hipStream_t st) {
  switch (dtype) {
    case 0: return h_rows_t<cd, cd>(first, src, ld_src, n_src, dst, ld_dst, rows, N, perm, zeta, cs, st);
    case 1: return h_rows_t<cf, cf>(first, src, ld_src, n_src, dst, ld_dst, rows, N, perm, zeta, cs, st);
    case 2: return h_rows_t<double, double>(first, src, ld_src, n_src, dst, ld_dst, rows, N, perm, zeta, cs, st);
    case 3: return h_rows_t<float, float>(first, src, ld_src, n_src, dst, ld_dst, rows, N, perm, zeta, cs, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace mn
