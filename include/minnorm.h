/*
 * minnorm.h -- C ABI of the MI355X (gfx950) randomized minimal-norm solver.
 *
 * Problem (Section 1; Section 4's setting): A is a full-rank m x n matrix with
 * m < n, b an m-vector and eps in (0, 1).  The solver returns x with
 * ||x - p|| <= eps ||p||, p being the minimal-Euclidean-norm solution of
 * A p = b.  The method is the paper's five steps with Steps 2-3 folded into
 * Step 4 (A c = b by Lemma 5.1, so Step 4's normal equations are A A* y = b):
 *   Step 1  S = T A*, T = S F D the l x N subsampled randomized Fourier
 *           transform (eqs. SRFT, SRFT2, randmat)          -> srft_sketch
 *   Step 2  Householder QR S = Q_S R, R kept                 -> build_preconditioner
 *   Step 4  preconditioned CG on A A* y = b, preconditioner R* R, stopped at
 *           Step 4's relative precision eps^2 l / (alpha N)  -> minnorm_solve
 *   Step 5  x = A* y (eq. output)                            -> minnorm_solve
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers (memory of the GPU current when
 *     the handle was created), except where a comment says "host".  The
 *     caller owns every buffer; the library never frees or keeps a caller
 *     pointer after the call returns.
 *   - Element types are selected by `dtype` (MN_C128 complex double,
 *     MN_C64 complex float, MN_F64 double, MN_F32 float).  Complex numbers
 *     are stored interleaved (re, im), as in C99 / C++ / numpy / torch.
 *   - A is row-major: entry (i, j) at A[i*lda + j], lda >= n.  Vectors are
 *     contiguous.  S and R are column-major: S(k, i) at S[k + i*lds].
 *   - N is the transform length, n <= N <= 2^22: a power of two, or N = N1 2^k
 *     with 2^k >= 256 and any N1 >= 2 (so any multiple of 256 from 512 up),
 *     since eq. (DFT) is defined for every length.  Such N keep the padding
 *     below 256 entries; their sketch runs only in the kept-outputs-only
 *     form (the l kept outputs of each row from N1 transforms of length 2^k),
 *     which holds l <= 2048 complex128 / float64 outputs per row at 256
 *     threads, 4096 at 512, and up to 8192 / 16384 for single precision; a
 *     larger l with such N is refused as an invalid N.  minnorm_steps23 and
 *     srft_sketch_noalloc take powers of two only.  Rows of A are
 *     zero-padded from n to N; this does not change the minimal-norm
 *     solution (its last N - n entries are zero).
 *   - d holds the N diagonal entries of D in FP64 whatever dtype is: complex
 *     unit-modulus phases (complex128) for complex dtypes, +-1 (float64) for
 *     real dtypes, where the transform F is the orthonormal discrete Hartley
 *     transform cas(2 pi j k / N) / sqrt(N) (the paper's real analogue).
 *     idx holds the l subsampled rows as int32: strictly increasing, in [0, N).
 *     The caller passes its own draw, or (minnorm_solve, minnorm_solve_batched)
 *     d = idx = NULL: the library then draws them itself as srft_draw
 *     defines, from mn_opts.seed, and redraws after a rank-deficient sketch.
 *   - Work is enqueued on the handle's stream.  Entry points that report a
 *     data-dependent status (rank deficiency, convergence, invalid idx)
 *     synchronise that stream before returning.
 *
 * Return values
 *    0  success
 *   -k  argument k (1-based position in the call) is invalid; nothing was
 *       enqueued.  For idx, validity is checked on the device: -k is then
 *       returned after a stream synchronisation, and no output is written.
 *   +1  MN_RANK_DEFICIENT: the sketch S is numerically rank-deficient
 *       (Remark 4.1): min_j |R_jj| <= tau max_i |R_ii|, tau = 16 sqrt(l) u
 *       for an FP64 sketch and 4 u for an FP32 one (u the unit roundoff).
 *       With a library draw this is returned only after mn_opts.max_reseed
 *       further independent draws (2 by default) were rank-deficient too
 *       (each draw fails with the small probability Lemma 3.1 bounds); with
 *       a caller's draw it is returned at once: redraw and call again.  A
 *       persistent +1 means A is not full rank.
 *   +2  MN_NOT_CONVERGED: the iteration cap was reached; x holds the last
 *       iterate and info the certificate reached.
 *   +3  MN_HIP_ERROR: a HIP runtime call failed (mn_last_hip_error()).
 *   +4  MN_NONFINITE: a non-finite value appeared (input or intermediate).
 */
#ifndef MINNORM_H
#define MINNORM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MN_OK 0
#define MN_RANK_DEFICIENT 1
#define MN_NOT_CONVERGED 2
#define MN_HIP_ERROR 3
#define MN_NONFINITE 4

enum mn_dtype { MN_C128 = 0, MN_C64 = 1, MN_F64 = 2, MN_F32 = 3 };

typedef struct mn_handle_s* mn_handle;

/* The optional factor H = Theta Pi Z Theta~ Pi~ Z~ of the SRFT (Section 3,
 * eqs. Rokhlin_trans and big_def), T = S F D H: device arrays of the caller.
 * Theta = R_1 R_2 ... R_{N-1}, R_k rotating coordinates (k-1, k) (zero-based)
 * by the block [[cos t_k, sin t_k], [-sin t_k, cos t_k]]; (Pi w)[j] =
 * w[perm[j]]; Z = diag(zeta). */
typedef struct {
  const double* theta;    /* [N-1] t_1 .. t_{N-1} of Theta (radians)            */
  const int32_t* perm;    /* [N] a permutation of 0 .. N-1                      */
  const void* zeta;       /* [N] unit-modulus complex128 (complex dtypes) or
                             +-1 float64 (real dtypes)                          */
  const double* theta_t;  /* the same for Theta~, Pi~, Z~                       */
  const int32_t* perm_t;
  const void* zeta_t;
} mn_hfactor;

/* Options of minnorm_solve / minnorm_solve_batched.  A NULL pointer or a zero
 * field selects the default given in brackets. */
typedef struct {
  double alpha;          /* alpha of Step 4's precision eps^2 l/(alpha N) [4]     */
  int32_t stop_rule;     /* 0: the paper's rule: f(y) - f* <= eps^2 l/(alpha N) f*,
                            certified from the CG scalars (the certificate rule
                            is used when l = N, where f* = 0);
                            1: the certificate rule ||x - p|| <= eps ||p||     [0] */
  int32_t max_iter;      /* cap on CG iterations (per refinement step)      [1000] */
  int32_t max_refine;    /* mixed precision: cap on FP64 refinement steps     [40] */
  int32_t check_every;   /* iterations enqueued between host reads of the
                            device stop flag; 0 = 2 for one right-hand side
                            (each read overlaps the next batch), 8 for the
                            block and batched forms                          [0] */
  int32_t inner_digits;  /* mixed precision: decimal digits each low-precision
                            inner solve gains; 0 = automatic: 3 where the
                            single-precision bulk accumulates in FP64 (the
                            factor's diagonal spans more than 3e4; a
                            refinement step then gains about two digits), else
                            4                                                [0] */
  int32_t block;         /* several right-hand sides: 0 = automatic (block form
                            when nrhs >= 2 and the bulk runs in single
                            precision), 1 = one right-hand side at a time,
                            2 = block form.  The block form runs the k CG
                            recurrences together: both products of an
                            iteration are split-BF16 matrix-core products
                            over all k columns (FP32 accumulation) and every
                            column is certified by FP64 refinement         [0] */
  int32_t streams;       /* minnorm_solve_batched: systems solved concurrently,
                            each on its own stream and host thread          [8] */
  int32_t precond;       /* source of Step 2's triangular factor R for the
                            solve: 0 = automatic: Cholesky of the FP64 Gram
                            matrix S* S (R* R = S* S for every QR of S), kept
                            when every pivot is positive and the diagonal of R
                            spans at most 1e5 (then R* R = S* S + E with
                            |E| <= c u64 |S|^2 leaves the preconditioned
                            operator within about 1e-6 of the identity),
                            otherwise the Householder factorisation;
                            1 = Householder QR of S always                  [0] */
  int32_t tune;          /* 1: a launch shape without a plan is timed over its
                            candidates on the live operands before use and the
                            fastest is kept in the handle's plan table (see
                            mn_plans_save); 0: plans already in the table, else
                            the built-in choices                            [0] */
  int32_t batch_form;    /* minnorm_solve_batched: 0 = fused when every system
                            has m <= 512 and precond = 0 (each stage of all
                            systems is one launch; the systems iterate in
                            lockstep, each with its own stopping test), else
                            concurrent lanes; 1 = concurrent lanes           [0] */
  int32_t refine;        /* 1: FP64 refinement around an FP64 bulk as well:
                            the inner CG runs on A itself to inner_digits and
                            the FP64 residual b - A A* y and x = A* y are
                            compensated once cond(A) u64 nears eps, as in the
                            mixed mode (the plain FP64 method's x = A* y has
                            a rounding floor of about cond(A) u64); 0 = FP64
                            refinement only around a single-precision bulk [0] */
  int32_t max_reseed;    /* library draw (d = idx = NULL): further draws after
                            a rank-deficient sketch before +1 is returned;
                            -1 = none, 0 = the default                        [2] */
  uint64_t seed;         /* library draw: the Philox key (see srft_draw)      [0] */
  int32_t graph;         /* minnorm_solve_batched's fused form: 0 or 1 = each
                            block of check_every lockstep iterations is
                            captured once as a HIP graph and replayed; -1 =
                            every kernel launched one by one                [0] */
  int32_t reserved;
  const mn_hfactor* hfactor;  /* host pointer: the SRFT's factor H (the sketch
                            is then S F D H applied to the rows); NULL = H = I,
                            the transform T = S F D.  Batched systems with H
                            run on the concurrent lanes                  [NULL] */
} mn_opts;

/* Per-solve report (host struct written by the library). */
typedef struct {
  int32_t status;        /* return value of this system                         */
  int32_t iters;         /* CG iterations, summed over refinement steps         */
  int32_t refine_steps;  /* FP64 residual evaluations (0 in plain FP64 mode)    */
  int32_t nrhs_done;     /* right-hand sides that met their stopping rule       */
  double cert_rel;       /* sqrt(rho / xi): the certificate of ||x-p|| / ||x||  */
  double rho0, rho, xi;  /* CG scalars at exit (see minnorm_solve)              */
  float stage_ms[8];     /* sketch, qr, cg, final product, refine, -, -, total  */
  int32_t retries;       /* library draw: redraws after a rank-deficient sketch
                            (the draw that was used has draw number retries) */
  int32_t factor;        /* Step 2's R: 1 = Cholesky of the FP64 Gram matrix
                            S* S, 2 = Householder QR of S                     */
  double kappa_hat;      /* lower estimate of cond(R) = cond(S): the larger of
                            max|R_ii| / min|R_ii| and, where the Gram route's
                            Cholesky ran through, the power-step estimate
                            sqrt(||R R*|| ||R^{-1} R^{-*}||) from 4 steps each;
                            it selects the Gram route (delta = sqrt(l) u64
                            kappa_hat^2 <= 0.1, or <= u32 kappa_hat for a
                            single-precision sketch; the plain solve's stopping
                            test then runs at eps sqrt(1 - delta)),
                            compensated residuals and FP64 accumulation of a
                            single-precision bulk                            */
} mn_info;

/* Handle: owns the stream binding and a device workspace reused across calls.
 * stream is a hipStream_t (NULL = the default stream).  Returns 0 or +3. */
int mn_create(mn_handle* h, void* stream);
int mn_destroy(mn_handle h);
int mn_set_stream(mn_handle h, void* stream);
const char* mn_status_string(int status);
const char* mn_last_hip_error(void);
/* Bytes of device workspace the handle currently holds. */
int64_t mn_workspace_bytes(mn_handle h);

/* Per-kernel timing for measurement (not part of the method).  With
 * enable = k > 0, every k-th later launch of each pass over A (k = 1: every
 * launch) is bracketed by a pair of HIP events on the handle's stream (each
 * pair adds a few microseconds between launches, hence the sampling);
 * enable <= 0 turns timing off.  mn_profile_read synchronises the
 * stream and returns how many launches of `kernel` ("gemv_adj": w = A* u,
 * "gemv_fwd": q = A w, "gram": the fused q = A (A* p) used when m <= 512,
 * "block_adj" / "block_fwd": the split-BF16 products W = A* P and Q = A W of
 * the multi-right-hand-side form, "block_residual": its FP64 products
 * U = A* Y and A U) were recorded since the last mn_profile call and their
 * summed duration in milliseconds.  Launches enqueued after the iteration
 * had already stopped (they return at once) are not counted.  mn_profile
 * clears the records.
 * Errors: -1 NULL handle; -2 unknown kernel name; -3/-4 NULL output. */
int mn_profile(mn_handle h, int enable);
int mn_profile_read(mn_handle h, const char* kernel, int64_t* count, double* total_ms);

/* Launch plans (autotuning).  A plan is one integer per kernel and shape:
 * "gram/<dtype>/<m>/<n>/<a>" fused pass (a = 1: single-precision data
 *                            accumulated in FP64): workgroup count (low 16 bits; 256,
 *                            512 or 1024), strip width (bit 16 set: 16
 *                            bytes of a row per thread instead of 32) and
 *                            strip order (bit 17 set: workgroup g takes strips
 *                            g, g + G, ... instead of a contiguous run) and
 *                            workgroup size (bit 18 set: 1024 threads, half
 *                            the rows per thread; 512 otherwise); bit 19 set:
 *                            the passes read a column-major copy of the bulk
 *                            matrix (m rounded up to 64, times n entries of
 *                            device workspace, kept by the handle), written by
 *                            the first pass of each solve with the other bits;
 *                            the default where the copy fits in half the free
 *                            device memory (else the row-major pass, 512);
 * "sketch_chunk_mb/<dtype>/<m>/<N>/0"  four-step FFT: MB of the intermediate
 *                            per chunk of rows (low 16 bits: 16 .. 512),
 *                            workgroup size in elements (bit 16 set: 2048,
 *                            else 4096), split (bits 17-18: N2 halved 0 .. 2
 *                            times), kept-outputs-only form (bits 19-20: 0
 *                            off, 1 / 2 / 3 for B = 16 / 8 / 4 columns per
 *                            block; applies for l <= 2048, or l <= 8192 for
 *                            single-precision data, else the full four-step
 *                            runs) with 2^(bits 21-24) column groups per row.
 *                            Default: that form with B = 16 and groups enough
 *                            for 512 workgroups where l <= 2048;
 * "gram_s/<dtype>/<m>/<l>/0"  Step 2's Gram matrix S* S: 0 on the FP64
 *                            matrix cores, 1 register-tiled on the vector
 *                            units (default 1 for m > 1024);
 * "block_fwd_wg/<dtype>/<m>/<n>/<k>"   block product A W: workgroups aimed
 *                            for when splitting its n columns (512..2048).
 * Plans are chosen by timing when mn_opts.tune = 1 (see there).
 * mn_plans_save writes the handle's table as JSON {"format":
 * "minnorm-plans-1", "plans": {key: value}, "best_ms": {key: ms}};
 * mn_plans_load merges such a file into the table (existing keys are
 * replaced).  mn_plans_count returns the number of plans held.
 * Errors: -1 NULL handle; -2 NULL path, unreadable/unwritable file or a file
 * without a "plans" object of "key": integer pairs. */
int mn_plans_save(mn_handle h, const char* path);
int mn_plans_load(mn_handle h, const char* path);
int mn_plans_count(mn_handle h);

/* Step 1, eq. (randmat): S = T A*, T = S F D of size l x N (eqs. SRFT,
 * SRFT2, with H = I), applied to every row of A:
 *   S(k, i) = (F (d o conj(a_i, zero-padded to N)))[idx[k]],  k < l, i < m,
 * F the unitary DFT of eq. (DFT) (real dtypes: the orthonormal Hartley
 * transform, no conjugation).
 *   A  [m x n, dtype, row-major, lda]      read
 *   d  [N, complex128 or float64]          read
 *   idx[l, int32]                          read
 *   S  [l x m, dtype, column-major, lds]   written
 * Errors: -3/-4 m, n < 1; -6 lda < n; -7 N not a transform length (see the
 * top of this file; also for (N, l) the kept-outputs-only form cannot hold),
 * N < n or N > 2^22; -8 l < 1 or l > N; -12 lds < l; -5/-9/-10/-11 NULL pointer;
 * -10 (after a sync) idx not strictly increasing or out of [0, N). */
int srft_sketch(mn_handle h, int dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                int64_t N, int64_t l, const void* d, const int32_t* idx,
                void* S, int64_t lds);

/* Steps 2-3 made explicit (Section 4, eqs. lineq and nonminnorm), a check
 * and export path beside minnorm_solve, which folds them into Step 4: with
 * S = T A* and its triangular factor R as the solve computes them,
 *   z = S R^{-1} R^{-*} b   the minimal-norm solution of S* z = b (eq. lineq)
 *   c = T* z                (eq. nonminnorm; c has N entries, the rows of A
 *                            being zero-padded to N)
 * By Lemma 5.1, A c = b (c's first n entries) and ||c|| = ||z||.
 *   A [m x n, dtype, row-major, lda]; b [m, FP64 wide type]; N, l, d, idx as
 *   in srft_sketch (m < l <= N)
 *   z [l, FP64 wide type (complex128 / float64)]  device, written
 *   c [N, FP64 wide type]                          device, written
 *   checks [3] optional host output: ||A c - b|| / ||b|| with A c summed in
 *   FP64 on the device, ||z||, ||c||.
 * Returns 0, +1 (rank-deficient sketch), +3, +4, or -k: -3 m < 1, m >= n or
 * m > 8192; -4 n; -5 A; -6 lda; -7 b; -8 N; -9 l <= m or l > N; -10 d;
 * -11 idx (also after a sync: not increasing in [0, N)); -12 z; -13 c. */
int minnorm_steps23(mn_handle h, int dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                    const void* b, int64_t N, int64_t l, const void* d, const int32_t* idx,
                    void* z, void* c, double* checks);

/* Step 1 with the paper's full transform T = S F D H (eq. SRFT with H of
 * eq. Rokhlin_trans): S(k, i) = (F (d o H conj(a_i)))[idx[k]] (real dtypes:
 * Hartley transform of d o H a_i).  H is applied to each row as two stages
 * (gather through the permutation times the phases, then the rotation chain
 * as a scan of affine maps) before the transform.  Arguments as srft_sketch,
 * with H (host struct of device arrays) at position 11.
 * Errors as srft_sketch (S, lds are -12, -13), and -11 for H NULL, an array
 * of it NULL, or (after a sync) a perm entry outside [0, N). */
int srft_sketch_h(mn_handle h, int dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                  int64_t N, int64_t l, const void* d, const int32_t* idx, const mn_hfactor* H,
                  void* S, int64_t lds);

/* srft_sketch without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, result and errors as srft_sketch, for
 * N <= 65536 (-7 beyond).  Its scratch (the twiddle table, the inverse
 * subsample map, the kept-output order with its twiddle table and the
 * four-step work area) lives in
 * a static device array of 32 MiB that the library holds on every GPU it
 * runs on until the process ends; the array's device address is looked up
 * once per device by mn_create.  Calls that overlap on one GPU (different
 * streams or handles) share that array and race; calls on one stream are
 * ordered.  The twiddle table is rebuilt when N or the precision changes.
 * Like srft_sketch, the call synchronises the stream once (idx's check). */
int srft_sketch_noalloc(mn_handle h, int dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                        int64_t N, int64_t l, const void* d, const int32_t* idx,
                        void* S, int64_t lds);

/* Step 1's random quantities (Section 3, eqs. SRFT, SRFT2: D's unit-modulus
 * phases, S's l rows sampled without replacement, as the paper's experiments
 * do), drawn with Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by
 * (seed mod 2^32, floor(seed / 2^32)); w(c0, c1, c2, c3) below is the four
 * output words at that counter.
 *   phases:  for j < N, with (x0, x1, x2, x3) = w(j, draw, 0, sys) and
 *            u = (floor(x0 / 2^5) 2^26 + floor(x1 / 2^6)) 2^-53 in [0, 1):
 *            complex dtypes d_j = exp(2 pi i u) (FP64), real dtypes
 *            d_j = 1 - 2 (x2 mod 2);
 *   indices: Floyd's sampling of l of N: for s = 0 .. l - 1 with
 *            t = N - l + s and (y0, y1, ..) = w(s, draw, 1, sys),
 *            r = floor((y0 2^32 + y1) (t + 1) / 2^64); the set gains r if r is
 *            not in it yet, else t.  idx = the set in increasing order.
 * minnorm_solve (sys = 0) and minnorm_solve_batched (sys = the system's
 * index) draw this way when given d = idx = NULL, with draw = 0 and then 1,
 * 2, ... for each redraw after a rank-deficient sketch.
 *   d   [N, complex128 for complex dtypes, float64 for real]  device, written
 *   idx [l, int32]                                           device, written
 * The phases are computed on the device; the indices on the host and copied
 * (the call returns after the copy has been enqueued and its host buffer
 * released, i.e. after a stream synchronisation).
 * Errors: -1 NULL handle; -2 dtype; -4 draw < 0; -5 sys < 0; -6 N < 1 or
 * N > 2^22; -7 l < 1 or l > N; -8 d NULL; -9 idx NULL. */
int srft_draw(mn_handle h, int dtype, uint64_t seed, int32_t draw, int32_t sys, int64_t N, int64_t l,
              void* d, int32_t* idx);

/* Step 2's factorisation: Householder QR of the l x m sketch, S = Q_S R
 * (tiled, blocked Householder reflections; Q_S is not formed).
 *   S [l x m, dtype, column-major, lds]  read
 *   R [m x m, dtype, column-major, ldr]  written: upper triangle = R with a
 *                                        real diagonal, strict lower = 0
 * R is unique up to a diagonal unitary factor.  Returns +1 when S is
 * numerically rank-deficient (Remark 4.1) -- R is still written.
 * Errors: -3 l < m; -4 m < 1; -5 NULL; -6 lds < l; -7 NULL; -8 ldr < m. */
int build_preconditioner(mn_handle h, int dtype, int64_t l, int64_t m,
                         const void* S, int64_t lds, void* R, int64_t ldr);

/* The whole method: x with ||x_j - p_j|| <= eps ||p_j|| for each of nrhs
 * right-hand sides b_j (Theorem 5.4; Step 4 is preconditioned CG on
 * A A* y = b stopped by opts->stop_rule; Step 5 x = A* y).
 *   A    [m x n, dtype, row-major, lda]  the problem matrix, read
 *   A_lo [m x n, row-major, lda_lo] optional copy of A in the single-precision
 *        type of the same kind (MN_C64 for MN_C128, MN_F32 for MN_F64), or
 *        NULL.  Given, the sketch, the QR and the bulk CG run on A_lo in FP32
 *        and FP64 iterative refinement on A (residual b - A A* y) restores the
 *        accuracy.  With dtype MN_C64 / MN_F32 the single-precision A is the
 *        problem itself: the bulk runs on it and the refinement residuals
 *        promote it exactly to FP64; A_lo must then be NULL.
 *   b    [nrhs x m, FP64 (complex128 / float64), b_j at b + j*ldb]   read
 *   N, l, d, idx: the SRFT's length and random quantities as in srft_sketch
 *        (m < l <= N; l = min(4m, N) is the paper's choice), or d = idx =
 *        NULL for the library's own draw (srft_draw with opts->seed, sys 0;
 *        redrawn up to opts->max_reseed times after a rank-deficient sketch,
 *        info->retries reports how many).
 *   x    [nrhs x n, FP64 (complex128 / float64), x_j at x + j*ldx]   written
 *   info optional host struct.
 * Errors: -2 dtype; -3 m < 1, m >= n or m > 8192; -4 n; -5 A; -6 lda; -7 A_lo with a
 * single-precision dtype; -8 lda_lo; -9 b; -10 ldb < m; -11 nrhs < 1 or > 64;
 * -12 eps not in (0,1); -13 N; -14 l <= m or l > N; -15 d NULL with idx
 * given; -16 idx NULL with d given, or (after a sync) not increasing in [0, N);
 * -17 opts field out of range; -18 x; -19 ldx < n. */
int minnorm_solve(mn_handle h, int dtype, int64_t m, int64_t n,
                  const void* A, int64_t lda, const void* A_lo, int64_t lda_lo,
                  const void* b, int64_t ldb, int64_t nrhs, double eps,
                  int64_t N, int64_t l, const void* d, const int32_t* idx,
                  const mn_opts* opts, void* x, int64_t ldx, mn_info* info);

/* Many independent systems of uneven sizes in one call.  Every array argument
 * below is a HOST array of `batch` entries; the pointers inside are device
 * pointers with the meaning of minnorm_solve (A_lo may be NULL, or hold NULL
 * entries: those systems then run in plain FP64).  A_lo[i] is read with
 * lda[i] as its leading dimension, the same as A[i].  b_i has m[i] entries,
 * x_i has n[i] entries; lda[i] >= n[i].  When some but not all A_lo entries
 * are NULL, every system runs on the concurrent lanes.  d and idx may both
 * be NULL (the arrays themselves): every system then uses the library's own
 * draw (srft_draw with opts->seed and sys = its index), with redraws as in
 * minnorm_solve.
 * info, if not NULL, is a host array of `batch` reports.  Returns the largest
 * status over the systems (each system's own status is in info[i].status).
 * Errors: -3 batch < 1; -4..-16 the matching array is NULL or an entry of it
 * is invalid as in minnorm_solve. */
int minnorm_solve_batched(mn_handle h, int dtype, int32_t batch,
                          const int64_t* m, const int64_t* n,
                          const void* const* A, const int64_t* lda,
                          const void* const* A_lo,
                          const void* const* b, const double* eps,
                          const int64_t* N, const int64_t* l,
                          const void* const* d, const int32_t* const* idx,
                          const mn_opts* opts, void* const* x, mn_info* info);

#ifdef __cplusplus
}
#endif

#endif /* MINNORM_H */
