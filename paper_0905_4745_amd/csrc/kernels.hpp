// Host-visible launch interfaces of the HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mn {

constexpr int kQrTile = 32;      // QR tile edge
constexpr int kFftMaxLds = 4096; // longest FFT done whole in one workgroup's LDS
constexpr int kMaxSlabs = 64;    // row slabs of the A* pass
constexpr int kMaxChunks = 256;  // column chunks of the A pass

inline int64_t dtype_size(int dtype) {
  switch (dtype) {
    case 0: return 16;
    case 1: return 8;
    case 2: return 8;
    case 3: return 4;
  }
  return 0;
}

struct FftPlan {
  int L;
  int nst;
  int radix[8];
};
FftPlan make_plan(int L);

struct SketchArgs {
  const void* A;
  int64_t lda, m, n, N, l;
  const void* d;        // FP64 phases (complex128) or signs (float64)
  const int32_t* idx;
  const int32_t* inv;   // inverse subsample map, N entries (four-step only)
  void* S;
  int64_t lds;
  const void* twiddle;  // W_N^k, k < N, in the compute precision
  void* work;           // four-step intermediate, chunk_rows * N complex
  int64_t chunk_rows;
};
hipError_t launch_sketch(int dtype, const SketchArgs& a, hipStream_t st);
int sketch_max_log2n(int dtype);  // largest log2(N) the four-step supports
hipError_t launch_inverse_map(const int32_t* idx, int64_t l, int64_t N, int32_t* inv, int32_t* bad, hipStream_t st);

struct QrArgs {
  const void* S;
  int64_t lds, l, m;
  void* R;
  int64_t ldr;
  void* work;       // qr_work_bytes
  double* diag_out; // [max |R_ii|, min |R_ii|, nonfinite flag]
};
int64_t qr_work_bytes(int dtype, int64_t l, int64_t m);
hipError_t launch_qr(int dtype, const QrArgs& a, hipStream_t st);

struct AdjArgs {
  const void* A;
  int64_t lda, m, n;
  const void* u;   // FP64, m entries
  void* w;         // n entries in the compute precision (may be null when w_wide set)
  void* w_wide;    // optional FP64 copy of w
  void* part;      // adj_part_elems(m, n) entries of the compute type
  const int32_t* flag;
};
int64_t adj_part_elems(int64_t m, int64_t n);
hipError_t launch_gemv_adj(int dtype, bool wide, const AdjArgs& a, hipStream_t st);

struct FwdArgs {
  const void* A;
  int64_t lda, m, n;
  const void* w;   // compute precision, n entries
  void* qpart;     // FP64, kMaxChunks * m
  const int32_t* flag;
  int* chunks_out;
};
hipError_t launch_gemv_fwd(int dtype, bool wide, const FwdArgs& a, hipStream_t st);

// CG state in device memory, written by the single-workgroup kernels.
struct PcgState {
  double rho0, rho, xi;
  double eps, alpha, l, N;
  double eps_outer, outer_rho, outer_xi;
  int32_t rule, max_iter, max_refine, status;
  int32_t iter_local, iter_total, refine_steps, done;
  int32_t outer_done, pad[3];
};

struct PcgVecs {
  const void* R;  // m x m, column-major, ldr, R's storage type
  int64_t ldr, m;
  const void* X;  // inverted diagonal blocks, FP64
  const void* b;  // right-hand side of the current solve (FP64)
  void *y, *r, *p, *z, *s, *q, *tv;  // FP64 m-vectors
  PcgState* state;
};
hipError_t launch_inv_diag(int rdtype, const void* R, int64_t ldr, int64_t m, void* X, hipStream_t st);
hipError_t launch_pcg_start(int rdtype, const PcgVecs& v, const void* parts, int nparts, const void* y_outer,
                            hipStream_t st);
hipError_t launch_pcg_tail(int rdtype, const PcgVecs& v, const void* qpart, int nparts, hipStream_t st);
hipError_t launch_refine_update(bool cplx, void* y_outer, const void* y, int64_t m, PcgState* state, hipStream_t st);

}  // namespace mn
