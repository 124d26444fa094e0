// Host-visible launch interfaces of the HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mn {

constexpr int kQrTile = 32;      // QR tile edge
constexpr int kFftMaxLds = 4096; // longest FFT done whole in one workgroup's LDS
constexpr int kMaxSlabs = 64;    // row slabs of the A* pass
constexpr int kMaxChunks = 256;  // column chunks of the A pass
constexpr int kMaxRows = 8192;   // largest m (the CG kernels keep an m-vector in LDS)

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
  int wg_elems;         // four-step: elements per workgroup (4096 or 2048; 0 = 4096)
  int split;            // four-step: N2 = 2^(floor(log2 N / 2) - split), split 0..2
  int pruned_b;         // > 0: kept outputs only, B = 16, 8 or 4 columns per block (N2 = 16 pruned_tpb / B)
  int pruned_ng;        // pruned: column groups per row (partial sums in work when > 1)
  int pruned_tpb;       // pruned: threads per workgroup (256, or sketch_pruned_wide_tpb: N2 = 16 tpb / B)
  int32_t* order;       // pruned: sketch_order_bytes(l) of scratch (kept outputs grouped by k mod N2, and
                        // their table of twiddle factors)
};
// column groups per row the pruned four-step uses for (B, ng), 0 if it does
// not apply to this (dtype, N, l); work then holds ng * chunk_rows * l
// elements of the compute type
int sketch_pruned_groups(int dtype, int64_t N, int64_t l, int B, int ng, int tpb = 256);
// bytes of the kept-outputs-only form's order buffer: l indices, then (from
// the next 256-byte boundary) 2 l entries of the compute type
int64_t sketch_order_bytes(int64_t l, bool single);
// the wide workgroup of the kept-outputs-only form (512 threads)
int sketch_pruned_wide_tpb(int dtype);
hipError_t launch_sketch(int dtype, const SketchArgs& a, hipStream_t st);
int sketch_max_log2n(int dtype);  // largest log2(N) the four-step supports
hipError_t launch_inverse_map(const int32_t* idx, int64_t l, int64_t N, int32_t* inv, int32_t* bad, hipStream_t st);
// The SRFT factor H = Theta Pi Z Theta~ Pi~ Z~ (hfactor.hip): rotation
// table cs (N pairs (cos, sin) of theta_k at index k), perm range check, and
// one stage "Theta Pi Z" on rows (first: the source is A, conjugated for
// complex data; else an earlier stage's rows, the result stored conjugated
// for complex data, ready for the sketch kernels).
hipError_t launch_h_rotations(const double* theta, int64_t N, double* cs, hipStream_t st);
hipError_t launch_h_check_perm(const int32_t* perm, int64_t N, int32_t* bad, hipStream_t st);
hipError_t launch_h_rows(int dtype, bool first, const void* src, int64_t ld_src, int64_t n_src, void* dst,
                         int64_t ld_dst, int64_t rows, int64_t N, const int32_t* perm, const void* zeta,
                         const double* cs, hipStream_t st);
// Steps 2-3 made explicit (steps23.hip): g = X* b and u = X g (X = R^{-1},
// FP64); z = S u with z scattered to y (N entries, zeroed before) at idx;
// d' = 1 and idx' = 0 .. N-1; c from the one-row transform t of y; the
// FP64 residual norms ||b - A c||^2, ||b||^2 from gemv_fwd chunk partials.
hipError_t launch_st_solve(bool cplx, const void* X, int64_t ldx, int64_t m, const void* b, void* g, void* u,
                           hipStream_t st);
hipError_t launch_st_z(int dtype, const void* S, int64_t lds, int64_t l, int64_t m, const void* u, const int32_t* idx,
                       void* z, void* y, hipStream_t st);
hipError_t launch_st_ones_iota(bool cplx, int64_t N, void* ones, int32_t* iota, hipStream_t st);
hipError_t launch_st_c(bool cplx, const void* t, const void* d, int64_t N, void* c, hipStream_t st);
hipError_t launch_st_resid(bool cplx, const void* qpart, int chunks, int64_t m, const void* b, double* out,
                           hipStream_t st);
// Twiddle table of the sketch (W_N^k, k < N, then the four-step splits'
// compact tables): twiddle_entries(N) complex entries of the compute precision.
int64_t twiddle_entries(int64_t N);
hipError_t launch_twiddles(bool single, int64_t N, void* out, hipStream_t st);
// Allocation-free sketch (noalloc.hip): a static device array of
// kNoAllocBytes per GPU, laid out as the twiddle table (kNoAllocTwBytes,
// enough for N <= kNoAllocMaxN), the inverse subsample map and the flag of
// idx's check, the kept-output order and table (sketch_order_bytes(l)), then
// the four-step work area.
constexpr int64_t kNoAllocBytes = (int64_t)32 << 20;
constexpr int64_t kNoAllocMaxN = 65536;
constexpr int64_t kNoAllocTwBytes = (int64_t)1152 << 10;   // >= twiddle_entries(65536) x 16 bytes
constexpr int64_t kNoAllocIdxBytes = kNoAllocMaxN * 4;      // inverse map
// device address of this device's array (set up by noalloc_init, which runs
// with the device current); null before
hipError_t noalloc_init(int device);
void* noalloc_ptr(int device);
// records that the twiddle region of `device` now holds table `tag`; true
// when it held another one (the caller then rebuilds it)
bool noalloc_twiddle_swap(int device, int64_t tag);
// The library's own draw of D and S (draw.hip): phases (complex128 or +-1
// float64, N entries) on the device, the l indices (increasing) on the host.
hipError_t launch_draw_phases(bool cplx, uint64_t seed, int draw, int sys, int64_t N, void* d, hipStream_t st);
// the phases of systems sys0 .. sys0 + count - 1 (count <= 65535; sys = the
// system's index) in one launch: tab (device) holds (N, byte offset from d)
// per system from system 0 on, max_n the largest N
hipError_t launch_draw_phases_batch(bool cplx, uint64_t seed, int draw, int sys0, int count, int64_t max_n,
                                    const int64_t* tab, void* d, hipStream_t st);
void draw_indices(uint64_t seed, int draw, int sys, int64_t N, int64_t l, int32_t* idx);

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
// out = [max |R_ii|, min |R_ii|, 1 if a diagonal entry is not finite]
hipError_t launch_rdiag_range(int dtype, const void* R, int64_t ldr, int64_t m, double* out, hipStream_t st);

struct AdjArgs {
  const void* A;
  int64_t lda, m, n;
  const void* u;   // FP64, m entries
  void* w;         // n entries in the compute precision (may be null when w_wide set)
  void* w_wide;    // optional FP64 copy of w
  void* part;      // adj_part_elems(m, n) entries of the compute type
  const int32_t* flag;
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;  // optional timing of the main kernel
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
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
};
hipError_t launch_gemv_fwd(int dtype, bool wide, const FwdArgs& a, hipStream_t st);
// Compensated (double-double accumulated) FP64 passes for the refinement:
// w = A* u (a.part holds adj_dd_part_elems(m, n) FP64 entries) and
// q = A w (a.qpart holds kMaxChunks * m entries; q receives the m sums and
// *a.chunks_out is set to 1).
int64_t adj_dd_part_elems(int64_t m, int64_t n);
hipError_t launch_gemv_adj_dd(int dtype, const AdjArgs& a, hipStream_t st);
hipError_t launch_gemv_fwd_dd(int dtype, const FwdArgs& a, void* q, hipStream_t st);

// Fused q = A (A* p) in one read of A (m <= kGramMaxRows, 16-byte aligned rows;
// up to kGramTallMaxRows from a column-major copy of A).
constexpr int kGramMaxRows = 512;
constexpr int kGramTallMaxRows = 2048;
constexpr int kGramMaxWg = 1024;  // partial sums per row (largest workgroup count)
constexpr int kGramParts = 1;    // slices of q left for the CG kernel to add
struct GramArgs {
  const void* A;
  int64_t lda, m, n;
  const void* p;   // FP64, m entries
  void* qpart;     // FP64, kGramMaxWg * m
  void* q;         // FP64, kGramParts * m: q = sum of the kGramParts slices
  const int32_t* flag;
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
  int max_wg = 512;  // plan: workgroups (each streams a contiguous run of strips)
  int narrow = 0;    // plan: strips of 16 bytes per thread and row instead of 32
  int interleave = 0;  // plan: workgroup g takes strips g, g + G, ... instead of a run
  int wide_wg = 0;     // plan: 1024 threads per workgroup (half the rows per thread)
  int wide_acc = 0;    // single-precision data: accumulate in FP64
  // column-major copy of A (column c at At + c ldt, ldt >= m): at_mode 1 =
  // the row-major pass that also writes it, 2 = the pass that reads it
  // instead of A
  void* At = nullptr;
  int64_t ldt = 0;
  int at_mode = 0;
  // m > kGramMaxRows: the pass over the column-major copy only (at_mode 1
  // writes the copy first, from A); shape code 0..3 (plan bits 20-21)
  int tall = 0;
};
bool gram_supported(int dtype, int64_t m, const void* A, int64_t lda);
// leading dimension of the column-major copy for m > kGramMaxRows: a
// multiple of this (rows m .. ldt - 1 of the copy are zero)
int64_t gram_tall_ld_multiple();
hipError_t launch_gram(int dtype, const GramArgs& a, hipStream_t st);
// Column-major copy At (ldt x n, ldt a multiple of 64 >= m, rows m .. ldt - 1
// zero) of a row-major m x n matrix of type dtype.
hipError_t launch_colmajor(int dtype, const void* A, int64_t lda, int64_t m, int64_t n, void* At, int64_t ldt,
                           hipStream_t st);
// The refinement residual's product q = A (A* y) in one compensated pass over
// the column-major copy At of the problem matrix (resid.hip), m <=
// kGramTallMaxRows; x_out (n, optional) receives A* y; part holds
// resid_part_elems(m, G) entries of the wide type.
int64_t resid_part_elems(int64_t m, int G);
hipError_t launch_resid_tall(int dtype, const void* At, int64_t ldt, int64_t m, int64_t n, const void* y, void* x_out,
                             void* part, int G, void* q, hipStream_t st);

// CG state in device memory, written by workgroup 0 of the CG kernels.
struct PcgState {
  double rho0, rho, rho_prev, xi;
  double eps, alpha, l, N;
  double eps_outer, outer_rho, outer_xi;
  int32_t rule, max_iter, max_refine, status;
  int32_t iter_local, iter_total, iter_snap, done;
  int32_t refine_steps, refine_snap, outer_done, pad;
};

// X = R^{-1} (FP64, column-major, leading dimension rinv_ld(m)).
int64_t rinv_ld(int64_t m);
hipError_t launch_rinv(int rdtype, const void* R, int64_t ldr, int64_t m, void* X, hipStream_t st);

// One CG step (see pcg.hip): start = 1 begins a solve from y = 0 with
// r = b - sum(parts) (parts may be null); start = 0 is an iteration with
// parts = the partial products of q = A A* p.
struct CgStep {
  const void* X;
  int64_t m;
  int start;
  const void* b;
  const void* parts;
  int nparts;
  void *p, *y;
  const void* r_in;
  void* r_out;
  void* s;
  const void* y_outer;  // start of an FP64 refinement step: certificate test
  PcgState* state;
};
hipError_t launch_cg_step(bool cplx, const CgStep& a, hipStream_t st);
hipError_t launch_refine_update(bool cplx, void* y_outer, const void* y, int64_t m, const PcgState* state,
                                hipStream_t st);
hipError_t launch_zero(bool cplx, void* v, int64_t m, hipStream_t st);

// ---- multi-right-hand-side block path (block.hip) ---------------------------
// Split-BF16 product C = L B^ (see block.hip): L as hi/lo planes (row-major,
// ld lda, Kp columns, Kp a multiple of bf_ktile()), B as compact hi/lo
// columns (kc of them, ld ldb).  mode 0: FP32 partials per split, mode 1:
// compact BF16 planes of C (one split).
struct BfGemmArgs {
  const uint16_t *Ahi, *Alo;
  int64_t lda, M;
  const uint16_t *Bhi, *Blo;
  int64_t ldb;
  int kc;
  int64_t Kp, ks;
  float* Cp;
  int64_t ldc;
  uint16_t *Ohi, *Olo;
  int64_t ldo;
  const int32_t* flag;
};
// FP64 product C = op(L) B^ with L of any dtype (see block.hip).
struct DGemmArgs {
  const void* A;
  int64_t lda, M, K;
  const void* B;
  int64_t ldb;
  int kc;
  int64_t ks;
  int tri;
  int herm;  // Gram product: skip tiles below the diagonal
  double* Cp;
  int64_t ldc;
  void* O;
  int64_t ldo;
  const int32_t* flag;
};
struct BlkCol {
  double rho0, rho, rho_prev, outer_rho, outer_xi;
  int32_t inner_done, outer_done, status, iters, refine, inner_it;
};
constexpr int kBlkMaxCols = 64;
struct BlkState {
  double eps_inner, eps_outer;
  int32_t kc, max_iter, max_refine, all_inner_done, all_outer_done, pad;
  BlkCol col[kBlkMaxCols];
};
int64_t bf_ktile();
int gemm_ncol(bool cplx, int kc);  // real output columns of a product with kc right-hand columns
hipError_t launch_planes(int dtype, const void* A, int64_t lda, int64_t M, int64_t K, bool trans, uint16_t* hi,
                         uint16_t* lo, int64_t ldp, hipStream_t st);
hipError_t launch_gemm_bf(bool cplx, bool conj, int mode, const BfGemmArgs& a, int splits, hipStream_t st);
hipError_t launch_gemm_d(int dtype, bool trans, bool conj, int mode, const DGemmArgs& a, int splits, hipStream_t st);
hipError_t launch_blk_reduce(bool cplx, bool f32, const void* Cp, int splits, int64_t ldc, int ncol, int64_t M,
                             int kc, const void* src, int64_t lds, void* out, int64_t ldo, const int32_t* flag,
                             hipStream_t st);
hipError_t launch_blk_outer(bool cplx, int kc, int64_t m, const void* b, int64_t ldb, const void* rr, const void* s,
                            const void* y_out, void* y, void* r, BlkState* state, hipStream_t st);
hipError_t launch_blk_alpha(bool cplx, int kc, int64_t m, const void* p, const void* q, void* y, void* r,
                            BlkState* state, hipStream_t st);
hipError_t launch_blk_beta(bool cplx, int kc, int64_t m, int start, const void* s, const void* z, void* p,
                           uint16_t* phi, uint16_t* plo, int64_t ldp, BlkState* state, hipStream_t st);
hipError_t launch_blk_flag(BlkState* state, hipStream_t st);
hipError_t launch_blk_refine(bool cplx, int kc, int64_t m, void* y_out, const void* y, BlkState* state,
                             hipStream_t st);
hipError_t launch_fill0(void* p, int64_t bytes, hipStream_t st);

// Preconditioner from the Gram matrix (chol.hip, block.hip): G = S* S in
// FP64, then R with R* R = G by blocked Cholesky (tiles of 32).
int gram_col_block(int dtype);
// G (FP64, upper triangle, ld ldg) = S* S on the vector units; with splits >
// 1 the K range is split in pieces of ks and Cp holds herk_part_elems(m,
// splits) FP64 (complex for complex data) partial entries.
int64_t herk_part_elems(int64_t m, int splits);
hipError_t launch_herk(int dtype, const void* S, int64_t lds, int64_t l, int64_t m, void* G, int64_t ldg, void* Cp,
                       int splits, int64_t ks, hipStream_t st);
// The same product on the FP64 matrix cores: 64 x 64 tiles of G, split K as
// launch_herk (same partial layout, herk_part_elems).
hipError_t launch_herk_mf(int dtype, const void* S, int64_t lds, int64_t l, int64_t m, void* G, int64_t ldg,
                          void* Cp, int splits, int64_t ks, hipStream_t st);
int herk_mf_tile();
hipError_t launch_gram_s(int dtype, const void* S, int64_t lds, int64_t l, int64_t m, void* G, int64_t ldg,
                         double* Cp, int64_t ldc, int splits, int64_t ks, hipStream_t st);
hipError_t launch_gram_fold(bool cplx, const double* Cp, int splits, int64_t ldc, int64_t m, void* G, int64_t ldg,
                            hipStream_t st);
// R (FP64, upper, ld ldr) from G (upper part, overwritten by Schur
// complements); Yd: chol_scratch_elems(m) FP64 entries (the inverses of the
// diagonal tiles); bad[0] = 1 if a pivot is not positive and finite.  With X
// (FP64, ld ldx >= rinv_ld(m)), X = R^{-1} on whole 32 x 32 blocks of the
// upper block triangle as well (lower blocks untouched).
int64_t chol_scratch_elems(int64_t m);
hipError_t launch_chol(bool cplx, void* G, int64_t ldg, int64_t m, void* R, int64_t ldr, void* Yd, void* X,
                       int64_t ldx, int32_t* bad, hipStream_t st);
// Power steps on T T* for two upper triangular FP64 matrices T0, T1 (ld0,
// ld1) at once: out[t * steps + k] (k < steps) = ||T_t T_t* v_k|| with v_0 a
// fixed unit vector and v_{k+1} the normalised product; each is a lower
// bound of sigma_max(T_t)^2.  work: power_work_elems(m) entries (wide).
int64_t power_work_elems(int64_t m);
hipError_t launch_power_sq(bool cplx, const void* T0, int64_t ld0, const void* T1, int64_t ld1, int64_t m, void* work,
                           double* out, int steps, hipStream_t st);

// ---- batched systems -----------------------------------------------------------
// Batched launch over several systems: entry i holds system i's first
// workgroup (a prefix sum) and its own grid; entry nsys holds the total.  A
// system with no work in a launch has start[i] == start[i + 1].
struct BGrid {
  int32_t start, gx, gy, gz;
};

// One descriptor per system of minnorm_solve_batched's fused form: the
// caller's buffers, the system's launch parameters and its slice of the
// batch workspace.  Every batched kernel finds its system through a BGrid
// table (common.hpp) and runs the plain kernel's body on it.
struct BSys {
  const void* A;   // problem data (FP64 residuals, x = A* y)
  int64_t lda;
  const void* Ab;  // bulk copy (the sketch and the inner iterations)
  int64_t ldab;
  int64_t m, n, N, l;
  const void* b;   // FP64 right-hand side (wide type)
  void* x;         // FP64 solution (wide type)
  const void* d;
  const int32_t* idx;
  // sketch plan: small FFT (N in LDS): pl_a = plan(N), fft_ba transforms per
  // workgroup; four-step: pl_a = plan(N1) with fft_ba (rows pass), pl_b =
  // plan(N2) with fft_bb (columns pass)
  FftPlan pl_a, pl_b;
  int fft_ba, fft_bb, N1, N2;
  int sk_kpt;      // kept-outputs-only four-step: accumulators per thread (2, 4, 8), or 0
  int32_t* order;  // sketch_order_bytes(l): kept outputs grouped by k mod N2 (kept-outputs-only form)
  const void* tw;  // W_N^k, k < N, compute precision
  // workspace
  int32_t* inv;    // N
  int32_t* flags;  // [0] idx invalid, [1] Cholesky pivot not positive
  void* S;         // l x m, bulk dtype, column-major
  void* Y;         // four-step intermediate, m x N (compute precision, complex)
  void* G;         // m x m, wide
  void* R;         // m x m, wide
  void* X;         // ldx x ldx, wide
  int64_t ldx;
  void* Yd;        // chol_scratch_elems(m), wide (inverses of R's diagonal tiles)
  double* diag;    // [max |R_ii|, min |R_ii|, nonfinite, power records of R R* times X X*]
  void* pw;        // 3 m, wide (power-step vectors)
  void *y, *r0, *r1, *p, *s, *q, *qpart, *w64, *apart, *fpart, *y_outer;
  PcgState* st;
  int64_t gram_spw, gram_nstrips;
  int gram_G;
  void* At;        // column-major copy of Ab for the fused pass (ldt x n), or null
  int64_t ldt;
  int64_t cm_spw, cm_nstrips;  // strips of the pass over At
  int64_t res_spw, res_nstrips;  // strips of the FP64 residual pass over A
  int adj_slabs;
  int64_t adj_rps;
  int fwd_chunks;
  int64_t fwd_chunk;
};
struct BLaunch {
  const BSys* sys;   // device array
  const BGrid* grid; // device array of nsys + 1
  int nsys;
  int total;         // workgroups (grid[nsys].start)
};
// per-system grids (host) for the passes whose shapes depend on the data
// (pruned: the kept-outputs-only four-step, one workgroup per row; s.sk_kpt
// is then its accumulator class 2, 4 or 8, else 0)
void b_plan_sketch(int dtype, BSys& s, BGrid& small, BGrid& cols, BGrid& rows, BGrid& pruned, size_t& lds_small,
                   size_t& lds_cols, size_t& lds_rows, size_t& lds_pruned);
// Y entries (0 for the small FFT and the kept-outputs-only form)
int64_t b_sketch_work_elems(int dtype, int64_t m, int64_t N, int64_t l);
// returns the rows-per-thread class (0..3: m <= 64, 128, 256, 512)
int b_plan_gram(int bulk_dtype, BSys& s, BGrid& gram, BGrid& gram_red);
void b_plan_wide(int dtype, bool aligned, BSys& s, BGrid& adj, BGrid& sum, BGrid& fwd);
bool b_aligned16(const void* p, int64_t ld, int dtype);
hipError_t launch_b_prep(const BLaunch& fill, const BLaunch& map, hipStream_t st);
// pruned[c]: the kept-outputs-only launches of accumulator class c (2, 4, 8
// kept outputs per thread); order: one 1024-thread workgroup per system
hipError_t launch_b_sketch(int dtype, const BLaunch& small, const BLaunch& cols, const BLaunch& rows,
                           const BLaunch& order, const BLaunch* pruned, size_t lds_small, size_t lds_cols,
                           size_t lds_rows, size_t lds_pruned, hipStream_t st);
hipError_t launch_b_gram_s(int dtype, const BLaunch& L, hipStream_t st);
hipError_t launch_b_chol_step(bool cplx, const BLaunch& L, int k, hipStream_t st);
// diag[3] = (power record of R R*) x (power record of X X*), steps power
// steps each (launch_power_sq's records), one workgroup per system; reads R
// and X = R^{-1}, uses pw
hipError_t launch_b_power(bool cplx, const BLaunch& L, int steps, hipStream_t st);
hipError_t launch_b_rdiag(bool cplx, const BLaunch& L, hipStream_t st);
hipError_t launch_b_inv_diag(bool cplx, const BLaunch& L, hipStream_t st);
hipError_t launch_b_trtri_step(bool cplx, const BLaunch& L, int k, hipStream_t st);
// the fused pass q = A (A* p) on the bulk copy (16-byte aligned rows), one
// launch per rows-per-thread class L[0..3], then the partial sums
// mode 0: row-major pass over Ab; 1: the same, also writing each system's
// column-major copy At (never skipped); 2: the pass over At
// side streams and events that let the rows-per-lane classes of a batched
// pass run concurrently (fork from and join back into the calling stream)
struct StreamFork {
  hipStream_t side[3];
  hipEvent_t ev[4];
};
hipError_t launch_b_gram(int dtype, const BLaunch* L, const BLaunch& red, int mode, hipStream_t st,
                         const StreamFork* fk = nullptr);
// every system's column-major copy At (ldt) of its bulk matrix Ab; the
// system's grid is (ceil(n / b_colmajor_tw(dtype)), ldt / 64) tiles
hipError_t launch_b_colmajor(int dtype, const BLaunch& L, hipStream_t st);
int b_colmajor_tw(int dtype);
// the refinement's FP64 residual product q = A (A* y_outer) as one fused pass
// over each system's problem data A (dtype = the problem dtype); same grids
// as launch_b_gram, strips from b_plan_gram_res (after b_plan_gram)
hipError_t launch_b_gram_res(int dtype, const BLaunch* L, const BLaunch& red, hipStream_t st,
                             const StreamFork* fk = nullptr);
void b_plan_gram_res(int dtype, BSys& s);
// FP64 passes on the problem data: w64 (or x) = A* u, u = y_outer (outer) or y;
// fpart = A w64 in column chunks
hipError_t launch_b_adj_wide(int dtype, bool aligned, const BLaunch& L, const BLaunch& sum, int use_y, int to_x,
                             hipStream_t st);
hipError_t launch_b_fwd_wide(int dtype, bool aligned, const BLaunch& L, hipStream_t st);
// CG step: parts 0 none (start from r = b), 1 the FP64 chunks fpart, 2 the q slices
hipError_t launch_b_cg(bool cplx, const BLaunch& Ls, const BLaunch& Lp, int start, int parts, int outer, int par,
                       size_t lds, hipStream_t st);
hipError_t launch_b_refine(bool cplx, const BLaunch& L, hipStream_t st);
hipError_t launch_b_zero_outer(bool cplx, const BLaunch& L, hipStream_t st);

}  // namespace mn
