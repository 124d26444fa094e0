// C ABI of the solver (declared in include/minnorm.h): argument checks,
// device workspace, and the host drivers that enqueue the HIP kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <numeric>
#include <thread>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/minnorm.h"
#include "kernels.hpp"

using namespace mn;

namespace {

thread_local std::string g_last_hip_error;

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Twiddle {
  int64_t N = 0;
  void* p = nullptr;
};

}  // namespace

struct mn_handle_s {
  hipStream_t stream = nullptr;
  int device = 0;
  std::map<std::string, Buf> bufs;
  std::map<std::pair<int64_t, int>, Twiddle> tw;  // W_N^k tables by (N, single precision)
  PcgState* host_state = nullptr;  // pinned
  PcgState* host_snap = nullptr;   // pinned, 2 slots: state snapshots read back one batch late
  hipEvent_t snap_ev[2] = {};
  BlkState* host_blk = nullptr;    // pinned
  int32_t* host_flag = nullptr;    // pinned
  double* host_diag = nullptr;     // pinned, 32 doubles
  hipEvent_t ev[9] = {};
  bool events = false;
  // per-kernel timing (mn_profile): event pairs recorded around launches
  bool prof = false;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  int prof_every = 1;                       // bracket every prof_every-th launch
  int64_t prof_seen[8] = {};                // launches seen per kernel id
  struct ProfRec {
    int kid;      // kernel id
    size_t ev;    // index of the begin event in pool
    int64_t ord;  // launch ordinal of that kernel id
  };
  std::vector<ProfRec> recs;
  // concurrent lanes of minnorm_solve_batched: child handles on their own streams
  bool owns_stream = false;
  std::vector<mn_handle> lanes;
  // launch plans chosen by timing (mn_opts.tune), keyed by kernel and shape
  std::map<std::string, int> plans;
  std::map<std::string, float> plan_ms;
  hipEvent_t tev[2] = {};
  mn_handle parent = nullptr;  // lanes read and add plans through their parent
  double kappa_hat = 1.0;      // max|R_ii| / min|R_ii| of the last factorisation
  void* host_stage = nullptr;  // pinned staging of the fused batched form
  size_t host_stage_bytes = 0;
  int32_t* host_draw = nullptr;  // pinned staging of library-drawn indices
  size_t host_draw_n = 0;
  hipStream_t cap_stream = nullptr;  // records HIP graphs of the batched iteration blocks
  StreamFork fork{};                 // side streams of the batched passes' row classes
  bool fork_ready = false;
  hipEvent_t pre_ev[2] = {};         // fork and join of the early column-major copies
};

namespace {

struct HipFail {
  hipError_t e;
};

inline void ck(hipError_t e) {
  if (e != hipSuccess) throw HipFail{e};
}

void* ws(mn_handle h, const char* name, size_t bytes) {
  Buf& b = h->bufs[name];
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return b.p;
  if (b.p) {
    ck(hipStreamSynchronize(h->stream));
    ck(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  ck(hipMalloc(&b.p, bytes));
  b.bytes = bytes;
  return b.p;
}

bool is_pow2(int64_t N) { return N > 0 && (N & (N - 1)) == 0; }
// Transform lengths the sketch takes: powers of two, and N = N1 2^k (any N1
// >= 2, 2^k >= 256) through the kept-outputs-only form
bool is_fft_len(int64_t N) { return is_pow2(N) || (N >= 512 && N % 256 == 0); }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
bool is_complex(int dtype) { return dtype == MN_C128 || dtype == MN_C64; }
bool is_single(int dtype) { return dtype == MN_C64 || dtype == MN_F32; }
int compute_cplx_dtype(int dtype) { return is_single(dtype) ? 1 : 0; }  // twiddle table slot

// The sketch's twiddle table for (N, precision), built once per handle on the
// device (launch_twiddles) and kept.
const void* twiddles(mn_handle h, int64_t N, bool single) {
  Twiddle& t = h->tw[{N, single ? 1 : 0}];
  if (t.N == N && t.p) return t.p;
  ck(hipMalloc(&t.p, (size_t)(twiddle_entries(N) * (single ? 8 : 16))));
  ck(launch_twiddles(single, N, t.p, h->stream));
  t.N = N;
  return t.p;
}

int fail_hip(hipError_t e) {
  g_last_hip_error = hipGetErrorString(e);
  return MN_HIP_ERROR;
}

// kernel ids for mn_profile_read
enum { K_ADJ = 0, K_FWD = 1, K_GRAM = 2, K_BADJ = 3, K_BFWD = 4, K_DRES = 5 };
const char* kKernelNames[] = {"gemv_adj", "gemv_fwd", "gram", "block_adj", "block_fwd", "block_residual"};

// a begin/end event pair for one timed launch, or nulls when not profiling
// (or when this launch is not one of the sampled ones)
std::pair<hipEvent_t, hipEvent_t> prof_pair(mn_handle h, int kid) {
  if (!h->prof) return {nullptr, nullptr};
  const int64_t ord = h->prof_seen[kid]++;
  if (ord % h->prof_every != 0) return {nullptr, nullptr};
  while (h->pool.size() < h->pool_used + 2) {
    hipEvent_t e;
    ck(hipEventCreate(&e));
    h->pool.push_back(e);
  }
  const size_t i = h->pool_used;
  h->pool_used += 2;
  h->recs.push_back({kid, i, ord});
  return {h->pool[i], h->pool[i + 1]};
}

void ev_record(mn_handle h, int i) {
  if (h->events) (void)hipEventRecord(h->ev[i], h->stream);
}

// ---- launch plans -------------------------------------------------------------
// A plan is one integer per (kernel, dtype, shape) key.  With mn_opts.tune set,
// a key without a plan is decided by timing every candidate on the live
// operands (one warm-up launch, then the best of three, HIP events on the
// handle's stream); mn_plans_save / mn_plans_load keep the table as JSON.
// Lanes of the batched call share their parent's table.
std::mutex g_plan_mu;

mn_handle plan_owner(mn_handle h) { return h->parent ? h->parent : h; }

bool plan_find(mn_handle h, const std::string& key, int* v) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  mn_handle o = plan_owner(h);
  auto it = o->plans.find(key);
  if (it == o->plans.end()) return false;
  *v = it->second;
  return true;
}

template <typename F>
int plan_get(mn_handle h, const mn_opts& o, const std::string& key, const std::vector<int>& cands, F run) {
  int v = 0;
  if (plan_find(h, key, &v)) return v;
  if (!o.tune) return cands[0];
  float best = 1e30f;
  int pick = cands[0];
  for (int c : cands) {
    run(c);
    float tmin = 1e30f;
    for (int r = 0; r < 3; ++r) {
      ck(hipEventRecord(h->tev[0], h->stream));
      run(c);
      ck(hipEventRecord(h->tev[1], h->stream));
      ck(hipEventSynchronize(h->tev[1]));
      float t = 0.f;
      ck(hipEventElapsedTime(&t, h->tev[0], h->tev[1]));
      tmin = std::min(tmin, t);
    }
    if (tmin < best) {
      best = tmin;
      pick = c;
    }
  }
  std::lock_guard<std::mutex> lk(g_plan_mu);
  mn_handle ow = plan_owner(h);
  ow->plans[key] = pick;
  ow->plan_ms[key] = best;
  return pick;
}

std::string plan_key(const char* kind, int64_t a, int64_t b, int64_t c, int64_t d) {
  char buf[128];
  snprintf(buf, sizeof buf, "%s/%lld/%lld/%lld/%lld", kind, (long long)a, (long long)b, (long long)c, (long long)d);
  return buf;
}

// ----------------------------------------------------------------------------
// Step 1: sketch of the rows of A (dtype) into S (l x m, lds).  idx must
// already be validated into the inverse map `inv`.
// Caller-provided device memory for the sketch's scratch (the allocation-free
// entry point): the twiddle table, the kept-output order, and `work_bytes`
// bytes for the four-step intermediate or partial sums.
struct SketchArena {
  const void* twiddle;
  int32_t* order;
  void* work;
  int64_t work_bytes;
};

void run_sketch(mn_handle h, int dtype, int64_t m, int64_t n, const void* A, int64_t lda, int64_t N, int64_t l,
                const void* d, const int32_t* idx, const int32_t* inv, void* S, int64_t lds,
                const mn_opts* o = nullptr, const SketchArena* ar = nullptr, const mn_hfactor* H = nullptr);

// A length N that is not a power of two runs only in the kept-outputs-only
// form: some (B, workgroup) must apply to (N, l)
bool sketch_ok(int dtype, int64_t N, int64_t l) {
  if (is_pow2(N)) return true;
  if (!is_fft_len(N)) return false;
  for (int tpb : {256, sketch_pruned_wide_tpb(dtype)})
    for (int B : {16, 8, 4})
      if (sketch_pruned_groups(dtype, N, l, B, 1, tpb) > 0) return true;
  return false;
}

// Checks H's arrays (non-null, permutations in range; one stream sync).
bool hfactor_valid(mn_handle h, const mn_hfactor* H, int64_t N) {
  if (!H || !H->theta || !H->perm || !H->zeta || !H->theta_t || !H->perm_t || !H->zeta_t) return false;
  int32_t* bad = (int32_t*)ws(h, "h_bad", 16);
  ck(launch_fill0(bad, 16, h->stream));
  ck(launch_h_check_perm(H->perm, N, bad, h->stream));
  ck(launch_h_check_perm(H->perm_t, N, bad, h->stream));
  ck(hipMemcpyAsync(h->host_flag, bad, 4, hipMemcpyDeviceToHost, h->stream));
  ck(hipStreamSynchronize(h->stream));
  return *h->host_flag == 0;
}

// Step 1 with T = S F D H: H applied to chunks of rows (two stages into two
// N-wide row buffers), then the sketch of the transformed rows.
void run_sketch_h(mn_handle h, int dtype, int64_t m, int64_t n, const void* A, int64_t lda, int64_t N, int64_t l,
                  const void* d, const int32_t* idx, const int32_t* inv, void* S, int64_t lds, const mn_opts* o,
                  const mn_hfactor* H) {
  const int64_t es = dtype_size(dtype);
  double* cs = (double*)ws(h, "h_cs", (size_t)(N * 16));
  double* cs_t = (double*)ws(h, "h_cs_t", (size_t)(N * 16));
  ck(launch_h_rotations(H->theta, N, cs, h->stream));
  ck(launch_h_rotations(H->theta_t, N, cs_t, h->stream));
  // rows per chunk: 128 MB per buffer
  int64_t chunk = std::max<int64_t>(1, ((int64_t)128 << 20) / (N * es));
  chunk = std::min(chunk, m);
  void* T1 = ws(h, "h_rows1", (size_t)(chunk * N * es));
  void* T2 = ws(h, "h_rows2", (size_t)(chunk * N * es));
  for (int64_t r0 = 0; r0 < m; r0 += chunk) {
    const int64_t rows = std::min(chunk, m - r0);
    const void* Ar = (const char*)A + r0 * lda * es;
    ck(launch_h_rows(dtype, true, Ar, lda, n, T1, N, rows, N, H->perm_t, H->zeta_t, cs_t, h->stream));
    ck(launch_h_rows(dtype, false, T1, N, N, T2, N, rows, N, H->perm, H->zeta, cs, h->stream));
    run_sketch(h, dtype, rows, N, T2, N, N, l, d, idx, inv, (char*)S + r0 * lds * es, lds, o);
  }
}

void run_sketch(mn_handle h, int dtype, int64_t m, int64_t n, const void* A, int64_t lda, int64_t N, int64_t l,
                const void* d, const int32_t* idx, const int32_t* inv, void* S, int64_t lds,
                const mn_opts* o, const SketchArena* ar, const mn_hfactor* H) {
  if (H) {
    run_sketch_h(h, dtype, m, n, A, lda, N, l, d, idx, inv, S, lds, o, H);
    return;
  }
  const bool single = is_single(dtype);
  const int64_t ces = single ? 8 : 16;
  SketchArgs a{};
  a.A = A;
  a.lda = lda;
  a.m = m;
  a.n = n;
  a.N = N;
  a.l = l;
  a.d = d;
  a.idx = idx;
  a.inv = inv;
  a.S = S;
  a.lds = lds;
  a.twiddle = ar ? ar->twiddle : twiddles(h, N, single);
  const bool p2 = is_pow2(N);
  if (p2 && N <= kFftMaxLds) {
    ck(launch_sketch(dtype, a, h->stream));
    return;
  }
  // rows per four-step chunk: an intermediate of 64 MB by default (it can
  // stay in the 256 MB last-level cache between the two passes); the plan
  // picks 16 .. 512 MB (larger chunks give each launch more workgroups to
  // overlap loads with transforms)
  // plan: MB of intermediate per chunk (low 16 bits), bit 16 set: 2048
  // elements per workgroup instead of 4096, bits 17-18: four-step split,
  // bits 19-20: kept outputs only (pruned) with B = 16, 8, 4 columns per
  // block (codes 1, 2, 3; 0 = full four-step), bits 21-24: log2 of the
  // pruned form's column groups per row, bit 25: the pruned form's wide
  // workgroup (one per CU, N2 = 16 x its threads / B)
  static const int pruned_b[4] = {0, 16, 8, 4};
  const int wide_tpb = sketch_pruned_wide_tpb(dtype);
  auto run = [&](int pl) {
    const int mb = pl & 0xFFFF;
    a.wg_elems = (pl >> 16) & 1 ? 2048 : 4096;
    a.split = (pl >> 17) & 3;
    a.pruned_b = pruned_b[(pl >> 19) & 3];
    a.pruned_ng = 1 << ((pl >> 21) & 15);
    a.pruned_tpb = (pl >> 25) & 1 ? wide_tpb : 256;
    int64_t per_row = N;  // intermediate elements per row
    if (a.pruned_b) {
      const int ng = sketch_pruned_groups(dtype, N, l, a.pruned_b, a.pruned_ng, a.pruned_tpb);
      if (ng < 1) a.pruned_b = 0;  // not applicable to this shape: full four-step
      else per_row = ng > 1 ? (int64_t)ng * l : 0;
    }
    int64_t chunk = per_row > 0 ? ((int64_t)mb << 20) / (per_row * ces) : m;
    // the arena's work area bounds the chunk (one row always fits there)
    if (ar && per_row > 0) chunk = std::min<int64_t>(chunk, ar->work_bytes / (per_row * ces));
    if (chunk < 1) chunk = 1;
    if (chunk > m) chunk = m;
    a.chunk_rows = chunk;
    if (ar) {
      a.work = per_row > 0 ? ar->work : nullptr;
      a.order = a.pruned_b ? ar->order : nullptr;
    } else {
      a.work = per_row > 0 ? ws(h, "fft_y", (size_t)(chunk * per_row * ces)) : nullptr;
      a.order = a.pruned_b ? (int32_t*)ws(h, "sk_order", (size_t)sketch_order_bytes(l, single)) : nullptr;
    }
    ck(launch_sketch(dtype, a, h->stream));
  };
  // default: the pruned form with B = 16 for l <= 2048, with enough column
  // groups per row for 512 workgroups (two per CU).  For single-precision
  // sketches with 2048 < l <= 8192 it is a tuning candidate only: at
  // 2048 x 262144 (l = 8192) it measured no faster than the full four-step.
  // For larger l the wide form with B = 8 (N2 = 1024: half the outer sum of
  // B = 16), groups enough for 256 workgroups: at 2048 x 262144 complex64,
  // l = 8192, it measured 4.46 ms against 4.72 ms for B = 16 and 9.35 ms
  // for the full four-step; at 4096 x 131072, l = 16384, 6.99 ms.
  int mb = 64;
  if (!p2) {
    // N = N1 2^k: the first kept-outputs-only shape that applies, with
    // column groups enough for 256 workgroups
    mb = -1;
    for (int wide : {0, 1})
      for (int bc : {1, 2, 3}) {
        const int tpb = wide ? wide_tpb : 256;
        if (mb >= 0 || sketch_pruned_groups(dtype, N, l, pruned_b[bc], 1, tpb) < 1) continue;
        int lg = 0;
        while ((m << lg) < 256 && lg < 10 &&
               sketch_pruned_groups(dtype, N, l, pruned_b[bc], 1 << (lg + 1), tpb) == (1 << (lg + 1)))
          ++lg;
        mb = 64 | (bc << 19) | (lg << 21) | (wide << 25);
      }
    if (mb < 0) throw HipFail{hipErrorInvalidValue};
  } else if (l <= 2048 && sketch_pruned_groups(dtype, N, l, 16, 1) > 0) {
    int lg = 0;
    while ((m << lg) < 512 && lg < 10) ++lg;
    mb = 64 | (1 << 19) | (lg << 21);
  } else {
    for (int bc : {2, 1}) {
      if (sketch_pruned_groups(dtype, N, l, pruned_b[bc], 1, wide_tpb) < 1) continue;
      int lg = 0;
      while ((m << lg) < 256 && lg < 10 &&
             sketch_pruned_groups(dtype, N, l, pruned_b[bc], 1 << (lg + 1), wide_tpb) == (1 << (lg + 1)))
        ++lg;
      mb = 64 | (bc << 19) | (lg << 21) | (1 << 25);
      break;
    }
  }
  const std::string key = plan_key("sketch_chunk_mb", dtype, m, N, 0);
  if (o) {
    std::vector<int> cands{mb};
    if (p2) {
      for (int c : {64, 16, 32})
        if (c != mb) cands.push_back(c);
      for (int sp : {0, 1, 2})
        for (int c : {64, 128, 256, 512})
          if (sp || c != 64) cands.push_back((sp << 17) | c);
      cands.push_back(0x10000 | 512);
    }
    for (int wide : {0, 1})
      for (int bc : {1, 2, 3})
        for (int lg : {0, 1, 2, 3, 4})
          if (sketch_pruned_groups(dtype, N, l, pruned_b[bc], 1 << lg, wide ? wide_tpb : 256) == (1 << lg)) {
            const int c = 64 | (bc << 19) | (lg << 21) | (wide << 25);
            if (c != cands[0]) cands.push_back(c);
          }
    mb = plan_get(h, *o, key, cands, run);
  }
  else plan_find(h, key, &mb);
  run(mb);
}

// Validate idx on the device and build the inverse subsample map (in the
// handle's workspace, or in inv_buf / bad_buf when given).
bool prepare_idx(mn_handle h, const int32_t* idx, int64_t l, int64_t N, int32_t** inv_out,
                 int32_t* inv_buf = nullptr, int32_t* bad_buf = nullptr) {
  int32_t* inv = inv_buf ? inv_buf : (int32_t*)ws(h, "inv", (size_t)N * 4);
  int32_t* bad = bad_buf ? bad_buf : (int32_t*)ws(h, "bad", 16);
  ck(launch_inverse_map(idx, l, N, inv, bad, h->stream));
  ck(hipMemcpyAsync(h->host_flag, bad, 4, hipMemcpyDeviceToHost, h->stream));
  ck(hipStreamSynchronize(h->stream));
  *inv_out = inv;
  return *h->host_flag == 0;
}

// The library's own draw of D's phases (device) and S's indices (host, then
// copied through pinned memory); returns once the copy has left the staging
// buffer.
void draw_srft_into(mn_handle h, bool cplx, uint64_t seed, int draw, int sys, int64_t N, int64_t l, void* d,
                    int32_t* idx) {
  ck(launch_draw_phases(cplx, seed, draw, sys, N, d, h->stream));
  if (h->host_draw_n < (size_t)l) {
    if (h->host_draw) {
      ck(hipStreamSynchronize(h->stream));
      ck(hipHostFree(h->host_draw));
      h->host_draw = nullptr;
      h->host_draw_n = 0;
    }
    ck(hipHostMalloc((void**)&h->host_draw, (size_t)l * sizeof(int32_t), hipHostMallocDefault));
    h->host_draw_n = (size_t)l;
  }
  draw_indices(seed, draw, sys, N, l, h->host_draw);
  ck(hipMemcpyAsync(idx, h->host_draw, (size_t)l * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  ck(hipStreamSynchronize(h->stream));
}

// The same for several systems (draw 0, sys = the system's index): every
// system's phases are launched, all index sets are drawn into one pinned
// buffer and copied, and the stream is synchronised once.
int64_t a256(int64_t v) { return (v + 255) / 256 * 256; }

// the handle's fork for the batched passes, created on first use (default
// priority, non-blocking streams; events without timing)
const StreamFork* handle_fork(mn_handle h) {
  if (!h->fork_ready) {
    for (auto& sd : h->fork.side)
      if (!sd) ck(hipStreamCreateWithFlags(&sd, hipStreamNonBlocking));
    for (auto& e : h->fork.ev)
      if (!e) ck(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto& e : h->pre_ev)
      if (!e) ck(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->fork_ready = true;
  }
  return &h->fork;
}

// The library's draws for systems 0 .. batch - 1 (draw 0, sys = the
// system's index) into contiguous device areas: system i's phases at
// dbase + doff[i] bytes, its indices at ibase + ioff[i] bytes, with
// doff/ioff the running sums of a256(N es) and a256(4 l).  The phases take
// one launch (its table of (N, offset) goes first, through the pinned
// staging buffer), the index sets are drawn meanwhile on host threads and
// leave in one copy; returns once the staging buffer is free again.
void draw_srft_batch(mn_handle h, bool cplx, uint64_t seed, int batch, const int64_t* N, const int64_t* l,
                     void* dbase, int32_t* ibase, int64_t* tab_dev) {
  const int64_t es = cplx ? 16 : 8;
  std::vector<int64_t> ioff((size_t)batch + 1, 0);
  int64_t doff = 0, max_n = 0;
  for (int i = 0; i < batch; ++i) ioff[i + 1] = ioff[i] + a256(l[i] * 4);
  // staging: the table (2 batch int64), then the index area
  const int64_t tab_bytes = a256(2 * (int64_t)batch * 8);
  const size_t need = (size_t)(tab_bytes + ioff[batch]);
  if (h->host_draw_n * sizeof(int32_t) < need) {
    if (h->host_draw) {
      ck(hipStreamSynchronize(h->stream));
      ck(hipHostFree(h->host_draw));
      h->host_draw = nullptr;
      h->host_draw_n = 0;
    }
    ck(hipHostMalloc((void**)&h->host_draw, need, hipHostMallocDefault));
    h->host_draw_n = need / sizeof(int32_t);
  }
  int64_t* tab = reinterpret_cast<int64_t*>(h->host_draw);
  for (int i = 0; i < batch; ++i) {
    tab[2 * i] = N[i];
    tab[2 * i + 1] = doff;
    doff += a256(N[i] * es);
    max_n = std::max(max_n, N[i]);
  }
  ck(hipMemcpyAsync(tab_dev, tab, (size_t)(2 * (int64_t)batch * 8), hipMemcpyHostToDevice, h->stream));
  for (int s0 = 0; s0 < batch; s0 += 65535)
    ck(launch_draw_phases_batch(cplx, seed, 0, s0, std::min(batch - s0, 65535), max_n, tab_dev, dbase, h->stream));
  char* hidx = reinterpret_cast<char*>(h->host_draw) + tab_bytes;
  const int nt = (int)std::max<unsigned>(1u, std::min<unsigned>(std::min(16u, std::thread::hardware_concurrency()),
                                                                   (unsigned)batch));
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t)
    pool.emplace_back([&, t]() {
      for (int i = t; i < batch; i += nt) draw_indices(seed, 0, i, N[i], l[i], (int32_t*)(hidx + ioff[i]));
    });
  for (int i = 0; i < batch; i += nt) draw_indices(seed, 0, i, N[i], l[i], (int32_t*)(hidx + ioff[i]));
  for (auto& th : pool) th.join();
  ck(hipMemcpyAsync(ibase, hidx, (size_t)ioff[batch], hipMemcpyHostToDevice, h->stream));
  ck(hipStreamSynchronize(h->stream));
}

// Redraws after a rank-deficient sketch when the library draws (max_reseed:
// 0 = the default 2, -1 = none).
int reseeds_of(const mn_opts& o) { return o.max_reseed == 0 ? 2 : (o.max_reseed < 0 ? 0 : o.max_reseed); }

// Step 2's factorisation; returns 0 or MN_RANK_DEFICIENT / MN_NONFINITE.
int run_qr(mn_handle h, int dtype, int64_t l, int64_t m, const void* S, int64_t lds, void* R, int64_t ldr) {
  QrArgs a{};
  a.S = S;
  a.lds = lds;
  a.l = l;
  a.m = m;
  a.R = R;
  a.ldr = ldr;
  a.work = ws(h, "qr", (size_t)qr_work_bytes(dtype, l, m));
  a.diag_out = (double*)ws(h, "qr_diag", 64);
  ck(launch_qr(dtype, a, h->stream));
  ck(hipMemcpyAsync(h->host_diag, a.diag_out, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  ck(hipStreamSynchronize(h->stream));
  const double mx = h->host_diag[0], mn_ = h->host_diag[1], nonfin = h->host_diag[2];
  h->kappa_hat = mn_ > 0.0 ? mx / mn_ : 1e300;
  if (nonfin != 0.0 || !std::isfinite(mx)) return MN_NONFINITE;
  // numerical rank test on the pivots: min |R_ii| >= sigma_min(R) and
  // max |R_ii| <= sigma_max(R), so a tiny ratio means a (nearly) singular
  // sketch.  FP32 sketches of ill-conditioned A legitimately reach ratios
  // near 1e-6, hence the tighter single-precision threshold.
  const double tau = is_single(dtype) ? 4.0 * 5.96e-8 : 16.0 * std::sqrt((double)l) * 1.11e-16;
  if (!(mn_ > tau * mx)) return MN_RANK_DEFICIENT;
  return MN_OK;
}

int64_t wide_size(int dtype) { return is_complex(dtype) ? 16 : 8; }

int64_t rup(int64_t a, int64_t b) { return cdiv(a, b) * b; }

// Step 2's triangular factor through the Gram matrix: G = S* S in FP64, R
// with R* R = G by blocked Cholesky (chol.hip).  Returns true with R64 (FP64,
// m x m, ld m) when every pivot is positive and finite and the factor is
// accurate enough; otherwise the caller uses the Householder factorisation
// (which also classifies rank deficiency and non-finite input).
//
// Accuracy: the computed R satisfies R* R = S* S + E with ||E|| about
// sqrt(l) u64 ||S||^2, so R^{-*} S* S R^{-1} is within delta = sqrt(l) u64
// cond(S)^2 of the identity, and sigma_min(A* R^{-1}) >= sqrt(1 - delta)
// (Step 4's bound sigma_min >= 1 for an exact R).  cond(S) = cond(R) is
// estimated from below by power steps on R R* and X X* (X = R^{-1}, both on
// the device) and by the diagonal spread; the larger of the two is
// kappa_hat.  The factor is kept when delta(kappa_hat) <= 0.1, or, for a
// single-precision sketch, when delta is no more than u32 kappa_hat: S's own
// rounding perturbs the preconditioned operator by that much whichever
// factorisation runs.  The plain solve's stopping test then runs at eps
// sqrt(1 - delta) (sigma_floor), which keeps its guarantee.
// the acceptance rule above, for a cond(S) estimate kap
double gram_delta(int64_t l, double kap) { return std::sqrt((double)l) * 1.11e-16 * kap * kap; }
bool gram_accurate(int64_t l, bool single_sketch, double kap) {
  const double tol = single_sketch ? std::max(0.1, 5.96e-8 * kap) : 0.1;
  return gram_delta(l, kap) <= tol;
}
// lower bound of sigma_min(A* R^{-1}) for a Gram-route R
double sigma_floor(int64_t l, double kap) { return std::sqrt(std::max(0.0, 1.0 - gram_delta(l, kap))); }

bool gram_factor(mn_handle h, int dtype, int64_t l, int64_t m, const void* S, int64_t lds, void* R64,
                 const mn_opts* o, void* X = nullptr, int64_t ldx = 0, double* kap_out = nullptr) {
  hipStream_t st = h->stream;
  const bool cplx = is_complex(dtype);
  const int64_t W = cplx ? 16 : 8;
  void* G = ws(h, "gram_G", (size_t)(m * m * W));
  // G = S* S: FP64 matrix-core product in the block GEMM's Hermitian mode
  // (plan 0), register-tiled FP64 product on the vector units (plan 1), or
  // the dedicated FP64 matrix-core Gram kernel (plan 2)
  auto run = [&](int pl) {
    if (pl == 2) {
      // split K so that the active tiles fill whole rounds of 1024
      // workgroups (four per CU) as nearly as possible
      const int64_t mt = cdiv(m, herk_mf_tile()), tiles = mt * (mt + 1) / 2;
      int best = 1;
      double best_eff = 0.0;
      for (int sp = 1; sp <= 8; ++sp) {
        if (sp > 1 && l / sp < 256) break;
        const double rounds = (double)(tiles * sp) / 1024.0;
        const double eff = rounds / std::ceil(rounds);
        if (eff > best_eff + 0.02) {
          best_eff = eff;
          best = sp;
        }
      }
      const int64_t ks = rup(cdiv(l, best), 16);
      const int splits = (int)cdiv(l, ks);
      void* Cp = splits > 1 ? ws(h, "herk_part", (size_t)(herk_part_elems(m, splits) * W)) : nullptr;
      ck(launch_herk_mf(dtype, S, lds, l, m, G, m, Cp, splits, ks, st));
      return;
    }
    if (pl == 1) {
      const int64_t tiles = std::max<int64_t>(1, cdiv(m, 128) * cdiv(m, 64) / 2);
      int64_t splits = std::min<int64_t>(std::min<int64_t>(std::max<int64_t>(cdiv(512, tiles), 1), 8), cdiv(l, 64));
      const int64_t ks = rup(cdiv(l, splits), 8);
      splits = cdiv(l, ks);
      void* Cp = splits > 1 ? ws(h, "herk_part", (size_t)(herk_part_elems(m, (int)splits) * W)) : nullptr;
      ck(launch_herk(dtype, S, lds, l, m, G, m, Cp, (int)splits, ks, st));
      return;
    }
    const int64_t nz = cdiv(m, gram_col_block(dtype));
    const int64_t tiles = cdiv(m, 128);
    const int64_t wgs = std::max<int64_t>(1, tiles * nz / 2 + 1);
    int64_t splits = std::min<int64_t>(std::max<int64_t>(cdiv(512, wgs), 1), cdiv(l, 64));
    const int64_t ks = rup(cdiv(l, splits), 16);
    splits = cdiv(l, ks);
    const int64_t ldc = rup(m, 4);
    double* Cp = nullptr;
    if (splits > 1) Cp = (double*)ws(h, "gram_part", (size_t)(nz * splits * 128 * ldc * 8));
    ck(launch_gram_s(dtype, S, lds, l, m, G, m, Cp, ldc, (int)splits, ks, st));
    if (splits > 1) ck(launch_gram_fold(cplx, Cp, (int)splits, ldc, m, G, m, st));
  };
  int pl = 2;
  const std::string key = plan_key("gram_s", dtype, m, l, 0);
  if (o) pl = plan_get(h, *o, key, {2, 1, 0}, run);
  else plan_find(h, key, &pl);
  run(pl);
  int32_t* bad = (int32_t*)ws(h, "chol_bad", 16);
  ck(launch_fill0(bad, 16, st));
  void* Yd = ws(h, "chol_yd", (size_t)(chol_scratch_elems(m) * W));
  ck(launch_chol(cplx, G, m, m, R64, m, Yd, X, ldx, bad, st));
  // dr[0..2]: the diagonal's range and non-finite count; dr[4..]: power
  // step records for R, then for X
  constexpr int kPow = 4;
  double* dr = (double*)ws(h, "qr_diag", (size_t)(4 + 2 * kPow) * 8);
  ck(launch_rdiag_range(cplx ? MN_C128 : MN_F64, R64, m, m, dr, st));
  ck(launch_fill0(dr + 4, 2 * kPow * 8, st));
  if (X != nullptr) ck(launch_power_sq(cplx, R64, m, X, ldx, m, ws(h, "cond_pw", (size_t)(power_work_elems(m) * W)), dr + 4, kPow, st));
  ck(hipMemcpyAsync(h->host_diag, dr, (size_t)(4 + 2 * kPow) * 8, hipMemcpyDeviceToHost, st));
  ck(hipMemcpyAsync(h->host_flag, bad, 4, hipMemcpyDeviceToHost, st));
  ck(hipStreamSynchronize(st));
  const double mx = h->host_diag[0], mn_ = h->host_diag[1], nonfin = h->host_diag[2];
  const double pr = h->host_diag[4 + kPow - 1], px = h->host_diag[4 + 2 * kPow - 1];
  double kap = mn_ > 0.0 ? mx / mn_ : 1e300;
  if (std::isfinite(pr) && std::isfinite(px) && pr > 0.0 && px > 0.0) kap = std::max(kap, std::sqrt(pr * px));
  else if (X != nullptr) kap = 1e300;
  h->kappa_hat = kap;
  if (kap_out) *kap_out = 0.0;
  if (*h->host_flag != 0 || nonfin != 0.0 || !std::isfinite(mx) || !(mn_ > 0.0)) return false;
  if (kap_out) *kap_out = kap;
  return gram_accurate(l, is_single(dtype), kap);
}


struct SolveCtx {
  mn_handle h;
  int dtype;      // problem dtype (A)
  int bulk;       // dtype of the matrix the CG bulk runs on
  bool mixed;     // FP64 refinement around a single-precision bulk
  const void* A;  // problem matrix
  int64_t lda;
  const void* Ab;  // bulk matrix
  int64_t ldab;
  int64_t m, n, N, l;
  double eps;
  mn_opts o;
  void* R;  // m x m, bulk dtype
  void* X;  // inverted diagonal blocks, FP64
  double sigma_lo = 1.0;  // lower bound of sigma_min(A* R^{-1}) (below 1 for a Gram-route R)
  bool comp = false;  // compensated FP64 refinement passes (cond(A) u64 near eps)
  bool wide_acc = false;  // single-precision bulk accumulated in FP64 (large cond(A))
  // column-major copies written on a side stream while Steps 1-2 ran (null
  // when not made): the bulk matrix's for the inner passes, the problem
  // matrix's for the compensated residuals; the solve's stream waits on
  // pre_ev before it reads them
  void* pre_at = nullptr;
  void* pre_res = nullptr;
  hipEvent_t pre_ev = nullptr;
};

void init_state(mn_handle h, PcgState* dst, const SolveCtx& c, int rule, double eps, int max_iter) {
  PcgState& s = *h->host_state;
  memset(&s, 0, sizeof(s));
  // rules 0 and 1 bound ||x - p|| by sqrt(rho) / sigma_min(A* R^{-1})
  s.eps = rule == 2 ? eps : eps * c.sigma_lo;
  s.alpha = c.o.alpha;
  s.l = (double)c.l;
  s.N = (double)c.N;
  s.eps_outer = c.eps;
  s.rule = rule;
  s.max_iter = max_iter;
  s.max_refine = c.o.max_refine;
  ck(hipMemcpyAsync(dst, &s, sizeof(PcgState), hipMemcpyHostToDevice, h->stream));
  // the staging struct is reused: wait until the copy has left it
  ck(hipStreamSynchronize(h->stream));
}

void read_state(mn_handle h, PcgState* src) {
  ck(hipMemcpyAsync(h->host_state, src, sizeof(PcgState), hipMemcpyDeviceToHost, h->stream));
  ck(hipStreamSynchronize(h->stream));
}

struct CgBufs {
  void *y, *r[2], *p, *s, *w, *part, *qpart, *q;
  PcgState* st;
  int par = 0;
  // column-major copy of the bulk matrix for the fused pass (written by the
  // first fused pass of the solve that uses it)
  void* at = nullptr;
  bool at_valid = false;
};

void cg_start(const SolveCtx& c, CgBufs& v, const void* b, const void* parts, int nparts, const void* y_outer) {
  CgStep a{};
  a.X = c.X;
  a.m = c.m;
  a.start = 1;
  a.b = b;
  a.parts = parts;
  a.nparts = nparts;
  a.p = v.p;
  a.y = v.y;
  a.r_in = nullptr;
  a.r_out = v.r[v.par];
  a.s = v.s;
  a.y_outer = y_outer;
  a.state = v.st;
  ck(launch_cg_step(is_complex(c.dtype), a, c.h->stream));
}

// CG iterations until the device flag is set (checked every check_every).
// Drop timing records of launches that found the stop flag set and returned
// at once: only the first `iters` launches of each kernel since the loop
// began (launch ordinals base[kid] on) did an iteration's work.
void prune_records(mn_handle h, size_t begin, const int64_t* base, int iters) {
  if (!h->prof) return;
  std::vector<mn_handle_s::ProfRec> kept(h->recs.begin(), h->recs.begin() + begin);
  for (size_t r = begin; r < h->recs.size(); ++r) {
    const auto& rec = h->recs[r];
    if (rec.ord - base[rec.kid] < iters) kept.push_back(rec);
  }
  h->recs.swap(kept);
}

void cg_loop(const SolveCtx& c, CgBufs& v, const void* b, int max_iter) {
  mn_handle h = c.h;
  const size_t rec_begin = h->recs.size();
  int64_t rec_base[8];
  std::copy(h->prof_seen, h->prof_seen + 8, rec_base);
  const int32_t* flag = &v.st->done;
  // One fused pass q = A (A* p).  plan: workgroup count (low 16 bits), bit 16
  // narrow strips, bit 17 interleaved strips, bit 18 1024 threads, bit 19:
  // read a column-major copy of A (the solve's first fused pass writes it,
  // with the row-major kernel and the other bits; it is never skipped by the
  // stop flag, so the copy is whole before any pass reads it).  For m above
  // kGramMaxRows (up to kGramTallMaxRows) only the pass over the copy exists
  // (bits 20-21: its shape code); the first pass of a solve then writes the
  // copy with a tiled transpose before reading it.
  const bool fused_rm = gram_supported(c.bulk, c.m, c.Ab, c.ldab);
  const bool tall = !fused_rm && c.m <= kGramTallMaxRows;
  int gram_plan = 512;
  const int64_t ldt = tall ? rup(c.m, gram_tall_ld_multiple()) : rup(c.m, 64);
  // the copy is taken only where it fits in half of the free device memory
  bool cm_ok = v.at != nullptr;
  if ((fused_rm || tall) && !cm_ok) {
    size_t fr = 0, tot = 0;
    cm_ok = hipMemGetInfo(&fr, &tot) == hipSuccess && (double)(ldt * c.n * dtype_size(c.bulk)) <= 0.5 * (double)fr;
  }
  const bool fused = fused_rm || (tall && cm_ok);
  auto gram = [&](int pl, const int32_t* flg, bool sampled) {
    if (!cm_ok) pl &= ~0x80000;
    if (tall) pl |= 0x80000;
    GramArgs ga{};
    ga.A = c.Ab;
    ga.lda = c.ldab;
    ga.m = c.m;
    ga.n = c.n;
    ga.p = v.p;
    ga.qpart = v.qpart;
    ga.q = v.q;
    ga.flag = flg;
    ga.max_wg = pl & 0xFFFF;
    ga.narrow = (pl >> 16) & 1;
    ga.interleave = (pl >> 17) & 1;
    ga.wide_wg = (pl >> 18) & 1;
    ga.wide_acc = c.wide_acc;
    ga.tall = (pl >> 20) & 3;
    if ((pl >> 19) & 1) {
      if (!v.at) v.at = ws(h, "gram_at", (size_t)(ldt * c.n * dtype_size(c.bulk)));
      ga.At = v.at;
      ga.ldt = ldt;
      if (!v.at_valid) {
        ga.at_mode = 1;
        ga.flag = nullptr;
        ck(launch_gram(c.bulk, ga, h->stream));
        v.at_valid = true;
        // not sampled (another kernel), but it takes its iteration's ordinal
        // so that the launches after the stop are still recognised
        if (sampled && h->prof) h->prof_seen[K_GRAM]++;
        return;
      }
      ga.at_mode = 2;
    }
    if (sampled) std::tie(ga.ev_begin, ga.ev_end) = prof_pair(h, K_GRAM);
    ck(launch_gram(c.bulk, ga, h->stream));
  };
  if (fused) {
    auto run = [&](int pl) { gram(pl, nullptr, false); };
    // default (first candidate): the column-major pass, 256 interleaved
    // workgroups, where the copy fits; else the row-major pass, 512
    std::vector<int> cands;
    if (tall) {
      // the pass over the copy: shape codes 0..3, 256 .. 1024 workgroups
      for (int code : {0, 1, 2, 3})
        for (int wg : {512, 256, 1024}) cands.push_back(wg | 0x80000 | (code << 20));
    } else {
      if (cm_ok)
        for (int il : {0x20000, 0})
          for (int wg : {256, 512, 1024}) cands.push_back(wg | il | 0x80000);
      for (int ww : {0, 0x40000})
        for (int il : {0, 0x20000})
          for (int nw : {0, 0x10000})
            for (int wg : {512, 256, 1024}) cands.push_back(wg | nw | il | ww);
    }
    gram_plan = plan_get(h, c.o, plan_key("gram", c.bulk, c.m, c.n, c.wide_acc ? 1 : 0), cands, run);
  }
  // the state is read one batch late (below), so short batches cost no idle
  // time and bound the launches enqueued after the stop
  const int ce = c.o.check_every > 0 ? c.o.check_every : 2;
  int enqueued = 0, snap = 0;
  bool pending = false;
  while (true) {
    for (int k = 0; k < ce; ++k) {
      if (fused) {
        gram(gram_plan, flag, true);
        CgStep a{};
        a.X = c.X;
        a.m = c.m;
        a.start = 0;
        a.b = b;
        a.parts = v.q;
        a.nparts = kGramParts;
        a.p = v.p;
        a.y = v.y;
        a.r_in = v.r[v.par];
        a.r_out = v.r[v.par ^ 1];
        a.s = v.s;
        a.state = v.st;
        ck(launch_cg_step(is_complex(c.dtype), a, h->stream));
        v.par ^= 1;
        continue;
      }
      AdjArgs aa{};
      aa.A = c.Ab;
      aa.lda = c.ldab;
      aa.m = c.m;
      aa.n = c.n;
      aa.u = v.p;
      aa.w = v.w;
      aa.part = v.part;
      aa.flag = flag;
      std::tie(aa.ev_begin, aa.ev_end) = prof_pair(h, K_ADJ);
      ck(launch_gemv_adj(c.bulk, c.wide_acc || !is_single(c.bulk), aa, h->stream));
      FwdArgs fa{};
      fa.A = c.Ab;
      fa.lda = c.ldab;
      fa.m = c.m;
      fa.n = c.n;
      fa.w = v.w;
      fa.qpart = v.qpart;
      fa.flag = flag;
      int chunks = 1;
      fa.chunks_out = &chunks;
      std::tie(fa.ev_begin, fa.ev_end) = prof_pair(h, K_FWD);
      ck(launch_gemv_fwd(c.bulk, c.wide_acc || !is_single(c.bulk), fa, h->stream));
      CgStep a{};
      a.X = c.X;
      a.m = c.m;
      a.start = 0;
      a.b = b;
      a.parts = v.qpart;
      a.nparts = chunks;
      a.p = v.p;
      a.y = v.y;
      a.r_in = v.r[v.par];
      a.r_out = v.r[v.par ^ 1];
      a.s = v.s;
      a.state = v.st;
      ck(launch_cg_step(is_complex(c.dtype), a, h->stream));
      v.par ^= 1;
    }
    enqueued += ce;
    // the state after this batch is copied back asynchronously and read one
    // batch later, so the host never leaves the stream idle while it checks
    // the stop flag; after the stop, the kernels of the batch still in
    // flight return at once and leave the state unchanged
    ck(hipMemcpyAsync(&h->host_snap[snap], v.st, sizeof(PcgState), hipMemcpyDeviceToHost, h->stream));
    ck(hipEventRecord(h->snap_ev[snap], h->stream));
    if (pending) {
      ck(hipEventSynchronize(h->snap_ev[snap ^ 1]));
      if (h->host_snap[snap ^ 1].done) {
        *h->host_state = h->host_snap[snap ^ 1];
        break;
      }
    }
    pending = true;
    snap ^= 1;
    if (enqueued > max_iter + 3 * ce) {  // cannot happen: the kernels cap iterations
      read_state(h, v.st);
      break;
    }
  }
  prune_records(h, rec_begin, rec_base, h->host_state->iter_local);
}

// One right-hand side; b and x FP64 device vectors.  Returns a status.
int solve_one(const SolveCtx& c, const void* b, void* x, mn_info* info) {
  mn_handle h = c.h;
  const int64_t W = wide_size(c.dtype);
  const int64_t m = c.m, n = c.n;
  CgBufs v;
  v.st = (PcgState*)ws(h, "state", sizeof(PcgState));
  v.y = ws(h, "y", m * W);
  v.r[0] = ws(h, "r0", m * W);
  v.r[1] = ws(h, "r1", m * W);
  v.p = ws(h, "p", m * W);
  v.s = ws(h, "s", m * W);
  v.w = ws(h, "w", (size_t)(n * W + 64));  // A* p in FP64
  v.part = ws(h, "adj_part", (size_t)(std::max(adj_part_elems(m, n), adj_dd_part_elems(m, n)) * W + 64));
  v.qpart = ws(h, "qpart", (size_t)((kMaxChunks > kGramMaxWg ? kMaxChunks : kGramMaxWg) * m * W));
  v.q = ws(h, "q", kGramParts * m * W);
  ev_record(h, 3);
  if (!c.mixed) {
    if (c.pre_ev) {
      // the copy written during Step 2
      ck(hipStreamWaitEvent(h->stream, c.pre_ev, 0));
      v.at = c.pre_at;
      v.at_valid = true;
    }
    init_state(h, v.st, c, c.o.stop_rule, c.eps, c.o.max_iter);
    cg_start(c, v, b, nullptr, 0, nullptr);
    cg_loop(c, v, b, c.o.max_iter);
    ev_record(h, 4);
    // Step 5: x = A* y
    AdjArgs aa{};
    aa.A = c.A;
    aa.lda = c.lda;
    aa.m = m;
    aa.n = n;
    aa.u = v.y;
    aa.w = x;
    aa.part = v.part;
    ck(launch_gemv_adj(c.dtype, true, aa, h->stream));
    ev_record(h, 5);
    read_state(h, v.st);
  } else {
    // FP64 refinement: r = b - A A* y_outer in FP64, inner CG in single
    // precision on the bulk copy, y_outer += dy, until the FP64 certificate
    // meets eps.
    void* y_outer = ws(h, "y_outer", m * W);
    void* qdd = ws(h, "q_dd", m * W);
    void* w64 = ws(h, "w64", (size_t)(n * W + 64));
    ck(launch_zero(is_complex(c.dtype), y_outer, m, h->stream));
    const double inner_eps = std::pow(10.0, -(double)c.o.inner_digits);
    init_state(h, v.st, c, 2, inner_eps, c.o.max_iter);
    // compensated residuals for m <= kGramTallMaxRows: one pass over a
    // column-major copy of the problem matrix (written once per solve, where
    // it fits in half the free memory) instead of an adjoint and a forward
    // pass; its column sums are x = A* y of the residual's y, kept for Step 5
    const int64_t rldt = rup(m, gram_tall_ld_multiple());
    bool fused_res = false;
    if (c.comp && m <= kGramTallMaxRows) {
      size_t fr = 0, tot = 0;
      fused_res = hipMemGetInfo(&fr, &tot) == hipSuccess &&
                  (double)(rldt * n * dtype_size(c.dtype)) <= 0.5 * (double)fr;
    }
    constexpr int kResG = 512;
    void* res_at = nullptr;
    void* res_x = nullptr;
    void* res_part = nullptr;
    if (c.pre_ev) {
      // the copies written during Steps 1-2 (the compensated residual serves
      // at any conditioning)
      ck(hipStreamWaitEvent(h->stream, c.pre_ev, 0));
      v.at = c.pre_at;
      v.at_valid = true;
      fused_res = true;
    }
    if (fused_res) {
      res_at = c.pre_res ? c.pre_res : ws(h, "res_at", (size_t)(rldt * n * dtype_size(c.dtype)));
      res_x = ws(h, "res_x", (size_t)(n * W + 64));
      res_part = ws(h, "res_part", (size_t)(resid_part_elems(m, kResG) * W));
      if (!c.pre_res) ck(launch_colmajor(c.dtype, c.A, c.lda, m, n, res_at, rldt, h->stream));
      // FP64 refinement around the FP64 matrix itself: the inner passes read
      // the same column-major copy (same leading dimension, zero padding)
      if (c.Ab == c.A && c.bulk == c.dtype && m > kGramMaxRows && rldt == rup(m, gram_tall_ld_multiple())) {
        v.at = res_at;
        v.at_valid = true;
      }
    }
    bool x_current = false;  // res_x holds A* y_outer of the current y_outer
    for (int outer = 0; outer <= c.o.max_refine + 1; ++outer) {
      AdjArgs aa{};
      aa.A = c.A;
      aa.lda = c.lda;
      aa.m = m;
      aa.n = n;
      aa.u = y_outer;
      aa.w = w64;
      aa.part = v.part;
      FwdArgs fa{};
      fa.A = c.A;
      fa.lda = c.lda;
      fa.m = m;
      fa.n = n;
      fa.w = w64;
      fa.qpart = v.qpart;
      int chunks = 1;
      fa.chunks_out = &chunks;
      if (outer == 0) {
        // y_outer = 0: the residual is b itself (no pass over A)
        cg_start(c, v, b, nullptr, 0, y_outer);
      } else if (fused_res) {
        ck(launch_resid_tall(c.dtype, res_at, rldt, m, n, y_outer, res_x, res_part, kResG, qdd, h->stream));
        x_current = true;
        cg_start(c, v, b, qdd, 1, y_outer);
      } else if (c.comp) {
        // b - A (A* y_outer) with double-double accumulation: the sums cancel
        // to about cond(A) times below their terms
        ck(launch_gemv_adj_dd(c.dtype, aa, h->stream));
        ck(launch_gemv_fwd_dd(c.dtype, fa, qdd, h->stream));
        cg_start(c, v, b, qdd, 1, y_outer);
      } else {
        ck(launch_gemv_adj(c.dtype, true, aa, h->stream));
        ck(launch_gemv_fwd(c.dtype, true, fa, h->stream));
        cg_start(c, v, b, v.qpart, chunks, y_outer);
      }
      read_state(h, v.st);
      if (h->host_state->outer_done) break;
      cg_loop(c, v, b, c.o.max_iter);
      ck(launch_refine_update(is_complex(c.dtype), y_outer, v.y, m, v.st, h->stream));
      x_current = false;
    }
    ev_record(h, 4);
    AdjArgs aa{};
    aa.A = c.A;
    aa.lda = c.lda;
    aa.m = m;
    aa.n = n;
    aa.u = y_outer;
    aa.w = x;
    aa.part = v.part;
    if (x_current) ck(hipMemcpyAsync(x, res_x, (size_t)(n * W), hipMemcpyDeviceToDevice, h->stream));
    else if (c.comp) ck(launch_gemv_adj_dd(c.dtype, aa, h->stream));
    else ck(launch_gemv_adj(c.dtype, true, aa, h->stream));
    ev_record(h, 5);
    read_state(h, v.st);
  }
  const PcgState& s = *h->host_state;
  int status = s.status;
  if (info) {
    info->iters += s.iter_total;
    info->refine_steps += s.refine_steps;
    if (status == MN_OK) info->nrhs_done += 1;
    const double rho = c.mixed ? s.outer_rho : s.rho;
    const double xi = c.mixed ? s.outer_xi : s.xi;
    const double cert = xi > 0 ? std::sqrt(rho / xi) : 0.0;
    if (cert > info->cert_rel) info->cert_rel = cert;
    info->rho0 = s.rho0;
    info->rho = rho;
    info->xi = xi;
  }
  return status;
}

// ----------------------------------------------------------------------------
// Multi-right-hand-side block path (see block.hip).  Columns are k
// independent CG recurrences on (A A*) y = b_j that share every pass over A:
// bulk products in split BF16, refinement residuals and the certificate in
// FP64, per-column stopping masks.  b, x FP64 (complex or real), ld ldb/ldx.
int64_t round_up(int64_t a, int64_t b) { return cdiv(a, b) * b; }

struct BlockPlan {
  int64_t Kp1, Kp2;          // K' extents of A* P (over rows) and A W (over columns)
  int s_fwd, s_d, s_res;     // splits of A W, of the X products, of A U
  int64_t ks_fwd, ks_d, ks_res;
  int64_t ldc;               // rows of a partial (m rounded to 4)
  int ncol;                  // real output columns
};

BlockPlan plan_block(bool cplx, int64_t m, int64_t n, int kc, int target_wg = 1024) {
  BlockPlan p{};
  const int64_t E = cplx ? 2 : 1;
  const int64_t kt = bf_ktile();
  p.Kp1 = round_up(E * m, kt);
  p.Kp2 = round_up(E * n, kt);
  p.ldc = round_up(m, 4);
  p.ncol = gemm_ncol(cplx, kc);
  const int64_t tiles = cdiv(m, 128);
  // about target_wg workgroups for the bulk product A W, 512 for the FP64 ones
  int64_t s = cdiv(target_wg, tiles);
  s = std::min<int64_t>(std::max<int64_t>(s, 1), p.Kp2 / kt);
  p.ks_fwd = round_up(cdiv(p.Kp2, s), kt);
  p.s_fwd = (int)cdiv(p.Kp2, p.ks_fwd);
  s = std::min<int64_t>(std::max<int64_t>(cdiv(512, tiles), 1), cdiv(m, 16));
  p.ks_d = round_up(cdiv(m, s), 16);
  p.s_d = (int)cdiv(m, p.ks_d);
  s = std::min<int64_t>(std::max<int64_t>(cdiv(512, tiles), 1), cdiv(n, 16));
  p.ks_res = round_up(cdiv(n, s), 16);
  p.s_res = (int)cdiv(n, p.ks_res);
  return p;
}

void read_blk(mn_handle h, BlkState* src) {
  ck(hipMemcpyAsync(h->host_blk, src, sizeof(BlkState), hipMemcpyDeviceToHost, h->stream));
  ck(hipStreamSynchronize(h->stream));
}

int solve_block(const SolveCtx& c, const void* b, int64_t ldb, int kc, void* x, int64_t ldx, mn_info* info) {
  mn_handle h = c.h;
  hipStream_t st = h->stream;
  const bool cplx = is_complex(c.dtype);
  const int64_t W = wide_size(c.dtype);
  const int64_t m = c.m, n = c.n;
  BlockPlan pl = plan_block(cplx, m, n, kc);
  const int64_t ldx_pre = rinv_ld(m);
  // bulk planes: A (m x Kp2) and its transpose (n x Kp1)
  uint16_t* a_hi = (uint16_t*)ws(h, "blk_a_hi", (size_t)(m * pl.Kp2 * 2));
  uint16_t* a_lo = (uint16_t*)ws(h, "blk_a_lo", (size_t)(m * pl.Kp2 * 2));
  uint16_t* t_hi = (uint16_t*)ws(h, "blk_t_hi", (size_t)(n * pl.Kp1 * 2));
  uint16_t* t_lo = (uint16_t*)ws(h, "blk_t_lo", (size_t)(n * pl.Kp1 * 2));
  if (c.pre_ev) {
    // written on the side stream during Step 2
    ck(hipStreamWaitEvent(st, c.pre_ev, 0));
  } else {
    ck(launch_planes(c.bulk, c.Ab, c.ldab, m, n, false, a_hi, a_lo, pl.Kp2, st));
    ck(launch_planes(c.bulk, c.Ab, c.ldab, m, n, true, t_hi, t_lo, pl.Kp1, st));
  }
  // right-operand planes (zero where the products never write)
  const size_t p_bytes = (size_t)(kc * pl.Kp1 * 2), w_bytes = (size_t)(kc * pl.Kp2 * 2);
  uint16_t* p_hi = (uint16_t*)ws(h, "blk_p_hi", p_bytes);
  uint16_t* p_lo = (uint16_t*)ws(h, "blk_p_lo", p_bytes);
  uint16_t* w_hi = (uint16_t*)ws(h, "blk_w_hi", w_bytes);
  uint16_t* w_lo = (uint16_t*)ws(h, "blk_w_lo", w_bytes);
  ck(launch_fill0(p_hi, (int64_t)p_bytes, st));
  ck(launch_fill0(p_lo, (int64_t)p_bytes, st));
  ck(launch_fill0(w_hi, (int64_t)w_bytes, st));
  ck(launch_fill0(w_lo, (int64_t)w_bytes, st));
  // block vectors, column-major with ld m
  const size_t vb = (size_t)round_up(kc * m * W, 16);
  void* yo = ws(h, "blk_yo", vb);
  void* y = ws(h, "blk_y", vb);
  void* rr = ws(h, "blk_rr", vb);
  void* r = ws(h, "blk_r", vb);
  void* p = ws(h, "blk_p", vb);
  void* q = ws(h, "blk_q", vb);
  void* s = ws(h, "blk_s", vb);
  void* z = ws(h, "blk_z", vb);
  // plan: workgroups of the A W product (split count over its n columns)
  {
    auto run = [&](int target) {
      const BlockPlan pp = plan_block(cplx, m, n, kc, target);
      float* qpt = (float*)ws(h, "blk_qp", (size_t)pp.s_fwd * pp.ncol * pp.ldc * 4);
      BfGemmArgs g2{};
      g2.Ahi = a_hi;
      g2.Alo = a_lo;
      g2.lda = pp.Kp2;
      g2.M = m;
      g2.Bhi = w_hi;
      g2.Blo = w_lo;
      g2.ldb = pp.Kp2;
      g2.kc = kc;
      g2.Kp = pp.Kp2;
      g2.ks = pp.ks_fwd;
      g2.Cp = qpt;
      g2.ldc = pp.ldc;
      ck(launch_gemm_bf(cplx, false, 0, g2, pp.s_fwd, st));
    };
    const int target = plan_get(h, c.o, plan_key("block_fwd_wg", c.bulk, m, n, kc), {1024, 512, 2048}, run);
    pl = plan_block(cplx, m, n, kc, target);
  }
  float* qp = (float*)ws(h, "blk_qp", (size_t)pl.s_fwd * pl.ncol * pl.ldc * 4);
  const int sd_max = std::max(pl.s_d, pl.s_res);
  double* dp = (double*)ws(h, "blk_dp", (size_t)sd_max * pl.ncol * pl.ldc * 8);
  BlkState* bst = (BlkState*)ws(h, "blk_state", sizeof(BlkState));
  ck(launch_fill0(yo, (int64_t)vb, st));
  for (int j = 0; j < kc; ++j) ck(hipMemsetAsync((char*)x + j * ldx * W, 0, (size_t)(n * W), st));
  {
    BlkState& hs = *h->host_blk;
    memset(&hs, 0, sizeof(hs));
    hs.eps_inner = std::pow(10.0, -(double)c.o.inner_digits);
    hs.eps_outer = c.eps;
    hs.kc = kc;
    hs.max_iter = c.o.max_iter;
    hs.max_refine = c.o.max_refine;
    ck(hipMemcpyAsync(bst, &hs, sizeof(BlkState), hipMemcpyHostToDevice, st));
    ck(hipStreamSynchronize(st));
  }
  const int32_t* inner_flag = &bst->all_inner_done;
  const int xdt = cplx ? MN_C128 : MN_F64;  // dtype of X = R^{-1} (FP64)

  // FP64 products with X: S = X* src (tri lower) or Z = X src (tri upper)
  auto x_product = [&](bool adjoint, const void* src, void* out, const int32_t* flag) {
    DGemmArgs g{};
    g.A = c.X;
    g.lda = ldx_pre;
    g.M = m;
    g.K = m;
    g.B = src;
    g.ldb = m;
    g.kc = kc;
    g.ks = pl.ks_d;
    g.tri = adjoint ? 2 : 1;
    g.Cp = dp;
    g.ldc = pl.ldc;
    g.flag = flag;
    // rows of X* are the stored columns of X; rows of X are read across them
    ck(launch_gemm_d(xdt, !adjoint, adjoint, 0, g, pl.s_d, st));
    ck(launch_blk_reduce(cplx, false, dp, pl.s_d, pl.ldc, pl.ncol, m, kc, nullptr, 0, out, m, flag, st));
  };

  ev_record(h, 3);
  for (int outer = 0; outer <= c.o.max_refine + 1; ++outer) {
    // FP64 residual of the current y_out: U = A* y_out (= x), rr = b - A U
    if (outer == 0) {
      ck(launch_blk_reduce(cplx, false, dp, 0, pl.ldc, pl.ncol, m, kc, b, ldb, rr, m, nullptr, st));
    } else {
      DGemmArgs g{};
      g.A = c.A;
      g.lda = c.lda;
      g.M = n;
      g.K = m;
      g.B = yo;
      g.ldb = m;
      g.kc = kc;
      g.ks = round_up(m, 16);
      g.O = x;
      g.ldo = ldx;
      auto ev = prof_pair(h, K_DRES);
      if (ev.first) ck(hipEventRecord(ev.first, st));
      ck(launch_gemm_d(c.dtype, true, true, 1, g, 1, st));
      if (ev.second) ck(hipEventRecord(ev.second, st));
      DGemmArgs f{};
      f.A = c.A;
      f.lda = c.lda;
      f.M = m;
      f.K = n;
      f.B = x;
      f.ldb = ldx;
      f.kc = kc;
      f.ks = pl.ks_res;
      f.Cp = dp;
      f.ldc = pl.ldc;
      ev = prof_pair(h, K_DRES);
      if (ev.first) ck(hipEventRecord(ev.first, st));
      ck(launch_gemm_d(c.dtype, false, false, 0, f, pl.s_res, st));
      if (ev.second) ck(hipEventRecord(ev.second, st));
      ck(launch_blk_reduce(cplx, false, dp, pl.s_res, pl.ldc, pl.ncol, m, kc, b, ldb, rr, m, nullptr, st));
    }
    x_product(true, rr, s, nullptr);
    ck(launch_blk_outer(cplx, kc, m, b, ldb, rr, s, yo, y, r, bst, st));
    ck(launch_blk_flag(bst, st));
    read_blk(h, bst);
    if (h->host_blk->all_outer_done) break;
    x_product(false, s, z, nullptr);
    ck(launch_blk_beta(cplx, kc, m, 1, s, z, p, p_hi, p_lo, pl.Kp1, bst, st));
    const size_t rec_begin = h->recs.size();
    int64_t rec_base[8];
    std::copy(h->prof_seen, h->prof_seen + 8, rec_base);
    while (true) {
      for (int it = 0; it < (c.o.check_every > 0 ? c.o.check_every : 8); ++it) {
        BfGemmArgs g1{};  // W = A* P (transposed planes, conjugated)
        g1.Ahi = t_hi;
        g1.Alo = t_lo;
        g1.lda = pl.Kp1;
        g1.M = n;
        g1.Bhi = p_hi;
        g1.Blo = p_lo;
        g1.ldb = pl.Kp1;
        g1.kc = kc;
        g1.Kp = pl.Kp1;
        g1.ks = pl.Kp1;
        g1.Ohi = w_hi;
        g1.Olo = w_lo;
        g1.ldo = pl.Kp2;
        g1.flag = inner_flag;
        auto ev = prof_pair(h, K_BADJ);
        if (ev.first) ck(hipEventRecord(ev.first, st));
        ck(launch_gemm_bf(cplx, true, 1, g1, 1, st));
        if (ev.second) ck(hipEventRecord(ev.second, st));
        BfGemmArgs g2{};  // Q = A W
        g2.Ahi = a_hi;
        g2.Alo = a_lo;
        g2.lda = pl.Kp2;
        g2.M = m;
        g2.Bhi = w_hi;
        g2.Blo = w_lo;
        g2.ldb = pl.Kp2;
        g2.kc = kc;
        g2.Kp = pl.Kp2;
        g2.ks = pl.ks_fwd;
        g2.Cp = qp;
        g2.ldc = pl.ldc;
        g2.flag = inner_flag;
        ev = prof_pair(h, K_BFWD);
        if (ev.first) ck(hipEventRecord(ev.first, st));
        ck(launch_gemm_bf(cplx, false, 0, g2, pl.s_fwd, st));
        if (ev.second) ck(hipEventRecord(ev.second, st));
        ck(launch_blk_reduce(cplx, true, qp, pl.s_fwd, pl.ldc, pl.ncol, m, kc, nullptr, 0, q, m, inner_flag, st));
        ck(launch_blk_alpha(cplx, kc, m, p, q, y, r, bst, st));
        x_product(true, r, s, inner_flag);
        x_product(false, s, z, inner_flag);
        ck(launch_blk_beta(cplx, kc, m, 0, s, z, p, p_hi, p_lo, pl.Kp1, bst, st));
      }
      read_blk(h, bst);
      if (h->host_blk->all_inner_done) break;
    }
    int live = 0;
    for (int j = 0; j < kc; ++j) live = std::max(live, h->host_blk->col[j].inner_it);
    prune_records(h, rec_begin, rec_base, live);
    ck(launch_blk_refine(cplx, kc, m, yo, y, bst, st));
  }
  ev_record(h, 4);
  ev_record(h, 5);
  read_blk(h, bst);
  const BlkState& hs = *h->host_blk;
  int worst = MN_OK;
  for (int j = 0; j < kc; ++j) {
    const BlkCol& col = hs.col[j];
    int status = col.status;
    if (!col.outer_done && status == MN_OK) status = MN_NOT_CONVERGED;
    worst = std::max(worst, status);
    if (info) {
      info->iters += col.iters;
      info->refine_steps += col.refine;
      if (status == MN_OK) info->nrhs_done += 1;
      const double cert = col.outer_xi > 0 ? std::sqrt(col.outer_rho / col.outer_xi) : 0.0;
      if (cert >= info->cert_rel) {
        info->cert_rel = cert;
        info->rho0 = col.rho0;
        info->rho = col.outer_rho;
        info->xi = col.outer_xi;
      }
    }
  }
  return worst;
}

mn_opts resolve_opts(const mn_opts* o) {
  mn_opts r{};
  if (o) r = *o;
  if (r.alpha == 0.0) r.alpha = 4.0;
  if (r.max_iter == 0) r.max_iter = 1000;
  if (r.max_refine == 0) r.max_refine = 40;
  // inner_digits 0 stays 0 (automatic): solve_impl decides once R is known
  if (r.streams == 0) r.streams = 8;
  return r;
}

bool opts_valid(const mn_opts& o) {
  return o.alpha > 1.0 && (o.stop_rule == 0 || o.stop_rule == 1) && o.max_iter > 0 && o.max_refine > 0 &&
         o.block >= 0 && o.block <= 2 && o.streams > 0 && o.streams <= 64 && (o.precond == 0 || o.precond == 1) &&
         (o.tune == 0 || o.tune == 1) && (o.batch_form == 0 || o.batch_form == 1) &&
         o.check_every >= 0 && o.check_every <= 1024 && o.inner_digits >= 0 && o.inner_digits <= 12 &&
         (o.refine == 0 || o.refine == 1) && o.max_reseed >= -1 && o.max_reseed <= 16 && o.graph >= -1 &&
         o.graph <= 1;
}

int solve_impl(mn_handle h, int dtype, int64_t m, int64_t n, const void* A, int64_t lda, const void* A_lo,
               int64_t lda_lo, const void* b, int64_t ldb, int64_t nrhs, double eps, int64_t N, int64_t l,
               const void* d, const int32_t* idx, const mn_opts& o, void* x, int64_t ldx, mn_info* info,
               int sys = 0) {
  SolveCtx c{};
  c.h = h;
  c.dtype = dtype;
  c.A = A;
  c.lda = lda;
  c.m = m;
  c.n = n;
  c.N = N;
  c.l = l;
  c.eps = eps;
  c.o = o;
  if (A_lo) {
    c.mixed = true;
    c.bulk = dtype + 1;  // C128 -> C64, F64 -> F32
    c.Ab = A_lo;
    c.ldab = lda_lo;
  } else if (is_single(dtype) || o.refine == 1) {
    // a single-precision problem, or FP64 refinement around the FP64 bulk
    c.mixed = true;
    c.bulk = dtype;
    c.Ab = A;
    c.ldab = lda;
  } else {
    c.mixed = false;
    c.bulk = dtype;
    c.Ab = A;
    c.ldab = lda;
  }
  if (info) {
    memset(info, 0, sizeof(*info));
  }
  h->events = info != nullptr;
  if (o.hfactor && !hfactor_valid(h, o.hfactor, N)) return -17;
  ev_record(h, 0);
  // the fused pass reads 16-byte vectors: an unaligned bulk row start is
  // re-laid once with a padded leading dimension (one pass over the bulk copy)
  if (m <= kGramMaxRows && !b_aligned16(c.Ab, c.ldab, c.bulk)) {
    const int64_t be = dtype_size(c.bulk);
    const int64_t pld = rup(n, std::max<int64_t>(16 / be, 1));
    void* pad = ws(h, "bulk_padded", (size_t)(pld * m * be));
    ck(hipMemcpy2DAsync(pad, (size_t)(pld * be), c.Ab, (size_t)(c.ldab * be), (size_t)(n * be), (size_t)m,
                        hipMemcpyDeviceToDevice, h->stream));
    c.Ab = pad;
    c.ldab = pld;
  }
  const int64_t bes = dtype_size(c.bulk);
  void* S = ws(h, "S", (size_t)(l * m * bes));
  const int wdt = is_complex(dtype) ? MN_C128 : MN_F64;
  int rdt = c.bulk;
  bool gram = false;
  // X = R^{-1}: built by the Cholesky launches on the Gram route, by its own
  // launches after the Householder factorisation otherwise
  const int64_t ldxi = rinv_ld(m);
  c.X = ws(h, "Xinv", (size_t)(ldxi * ldxi * wide_size(dtype)));
  const bool block = o.block == 2 || (o.block == 0 && nrhs >= 2 && c.mixed && is_single(c.bulk));
  // A single right-hand side of a refined solve with m in the tall form's
  // range: the column-major copies its passes read (of a separate
  // single-precision bulk for the inner passes, of the problem matrix for
  // the compensated residuals) are written on a side stream once the first
  // sketch is enqueued, overlapping Step 2 (matrix-core Gram product,
  // latency-bound Cholesky), where they fit in half the free memory
  // every way out of this call leaves the solve's stream behind the copies
  // (the next call may reuse or reallocate their buffers)
  struct PreJoin {
    mn_handle h;
    const hipEvent_t* e;
    ~PreJoin() {
      if (*e) (void)hipStreamWaitEvent(h->stream, *e, 0);
    }
  } pre_join{h, &c.pre_ev};
  auto start_copies = [&]() {
    // A plain solve whose fused pass reads the column-major copy (by the
    // stored launch plan) gets that copy the same way; its first pass then
    // reads the copy instead of writing it.
    int cm_plan = 0;
    if (!c.mixed && !block && nrhs == 1 && gram_supported(c.bulk, m, c.Ab, c.ldab) &&
        plan_find(h, plan_key("gram", c.bulk, m, n, 0), &cm_plan) && ((cm_plan >> 19) & 1)) {
      const int64_t cld = rup(m, 64);
      const size_t at_bytes = (size_t)(cld * n * dtype_size(c.bulk));
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess && (double)at_bytes <= 0.5 * (double)fr) {
        const StreamFork* fk = handle_fork(h);
        c.pre_at = ws(h, "gram_at", at_bytes);
        hipStream_t side = fk->side[0];
        ck(hipEventRecord(h->pre_ev[0], h->stream));
        ck(hipStreamWaitEvent(side, h->pre_ev[0], 0));
        ck(launch_colmajor(c.bulk, c.Ab, c.ldab, m, n, c.pre_at, cld, side));
        ck(hipEventRecord(h->pre_ev[1], side));
        c.pre_ev = h->pre_ev[1];
      }
      return;
    }
    // The block form's BF16 planes of the bulk matrix (and of its
    // transpose), the same way.
    if (block && is_single(c.bulk)) {
      const BlockPlan pl = plan_block(is_complex(dtype), m, n, (int)nrhs);
      uint16_t* a_hi = (uint16_t*)ws(h, "blk_a_hi", (size_t)(m * pl.Kp2 * 2));
      uint16_t* a_lo = (uint16_t*)ws(h, "blk_a_lo", (size_t)(m * pl.Kp2 * 2));
      uint16_t* t_hi = (uint16_t*)ws(h, "blk_t_hi", (size_t)(n * pl.Kp1 * 2));
      uint16_t* t_lo = (uint16_t*)ws(h, "blk_t_lo", (size_t)(n * pl.Kp1 * 2));
      const StreamFork* fk = handle_fork(h);
      hipStream_t side = fk->side[0];
      ck(hipEventRecord(h->pre_ev[0], h->stream));
      ck(hipStreamWaitEvent(side, h->pre_ev[0], 0));
      ck(launch_planes(c.bulk, c.Ab, c.ldab, m, n, false, a_hi, a_lo, pl.Kp2, side));
      ck(launch_planes(c.bulk, c.Ab, c.ldab, m, n, true, t_hi, t_lo, pl.Kp1, side));
      ck(hipEventRecord(h->pre_ev[1], side));
      c.pre_ev = h->pre_ev[1];
      return;
    }
    // (FP64 refinement around the FP64 matrix itself: one copy serves both)
    const bool sep = A_lo != nullptr;
    if (c.mixed && (sep || c.bulk == dtype) && !block && nrhs == 1 && m > kGramMaxRows &&
        m <= kGramTallMaxRows) {
      const int64_t tld = rup(m, gram_tall_ld_multiple());
      const size_t at_bytes = sep ? (size_t)(tld * n * dtype_size(c.bulk)) : 0;
      const size_t res_bytes = (size_t)(tld * n * dtype_size(dtype));
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess && (double)(at_bytes + res_bytes) <= 0.5 * (double)fr) {
        const StreamFork* fk = handle_fork(h);
        c.pre_res = ws(h, "res_at", res_bytes);
        c.pre_at = sep ? ws(h, "gram_at", at_bytes) : c.pre_res;
        hipStream_t side = fk->side[0];
        ck(hipEventRecord(h->pre_ev[0], h->stream));
        ck(hipStreamWaitEvent(side, h->pre_ev[0], 0));
        if (sep) ck(launch_colmajor(c.bulk, c.Ab, c.ldab, m, n, c.pre_at, tld, side));
        ck(launch_colmajor(dtype, A, lda, m, n, c.pre_res, tld, side));
        ck(hipEventRecord(h->pre_ev[1], side));
        c.pre_ev = h->pre_ev[1];
      }
    }
  };
  // Steps 1-2 for one draw of (d, idx): the caller's, or the library's own
  // (srft_draw), redrawn after a rank-deficient sketch (Remark 4.1)
  const bool lib_draw = d == nullptr;
  const int attempts = lib_draw ? 1 + reseeds_of(o) : 1;
  for (int att = 0;; ++att) {
    if (lib_draw) {
      void* dd = ws(h, "draw_d", (size_t)(N * (is_complex(dtype) ? 16 : 8)));
      int32_t* di = (int32_t*)ws(h, "draw_idx", (size_t)l * 4);
      draw_srft_into(h, is_complex(dtype), o.seed, att, sys, N, l, dd, di);
      d = dd;
      idx = di;
      if (info) info->retries = att;
    }
    int32_t* inv = nullptr;
    if (!prepare_idx(h, idx, l, N, &inv)) return -16;
    run_sketch(h, c.bulk, m, n, c.Ab, c.ldab, N, l, d, idx, inv, S, l, &o, nullptr, o.hfactor);
    // (after the compute-bound sketch, which holds every CU, so that the
    // copies share the chip with the Gram product and the Cholesky)
    if (!c.pre_ev) start_copies();
    ev_record(h, 1);
    // Step 2's R: Cholesky of the FP64 Gram matrix when that is accurate,
    // Householder QR of S otherwise
    rdt = c.bulk;
    gram = false;
    // the block products read whole tiles of X, so its strict lower part must be zero
    if (block) ck(launch_fill0(c.X, ldxi * ldxi * wide_size(dtype), h->stream));
    double kap_gram = 0.0;
    if (o.precond == 0) {
      c.R = ws(h, "R64", (size_t)(m * m * wide_size(dtype)));
      gram = gram_factor(h, c.bulk, l, m, S, l, c.R, &o, c.X, ldxi, &kap_gram);
      if (gram) rdt = wdt;
    }
    if (!gram) {
      c.R = ws(h, "R", (size_t)(m * m * bes));
      const int st = run_qr(h, c.bulk, l, m, S, l, c.R, m);
      // the Gram route's estimate (when its Cholesky ran through) stays a
      // lower bound of cond(S)
      h->kappa_hat = std::max(h->kappa_hat, kap_gram);
      if (st == MN_RANK_DEFICIENT && att + 1 < attempts) continue;
      if (st != MN_OK) {
        ev_record(h, 2);
        if (info) info->status = st;
        return st;
      }
    }
    break;
  }
  ev_record(h, 2);
  if (info) {
    info->factor = gram ? 1 : 2;
    info->kappa_hat = h->kappa_hat;
  }
  if (gram) c.sigma_lo = sigma_floor(l, h->kappa_hat);
  // compensated refinement passes when the rounding of plain FP64 sums,
  // about cond(A) u64 relative, is within a hundredth of eps
  c.comp = c.mixed && h->kappa_hat * 1.11e-16 > eps / 100.0;
  // single-precision sums over n terms carry about 1e-6 relative error; with
  // cond(A) above 3e4 the inner solves would stop contracting, so the bulk
  // passes then accumulate in FP64 (same bytes read)
  c.wide_acc = is_single(c.bulk) && h->kappa_hat > 3e4;
  // inner solves' precision, automatic: where the single-precision bulk is
  // that ill-conditioned, one refinement step gains about two digits however
  // far its inner solve goes (the single-precision copy's perturbation of
  // A A* limits it), so asking three wastes the fewest iterations (measured
  // at 2048 x 262144, cond 1e6: 2, 3, 4, 5, 6 digits took 74.7, 66.8, 75.8,
  // 84.0, 92.7 ms per solve); otherwise four
  if (c.o.inner_digits == 0) c.o.inner_digits = (c.wide_acc && !block) ? 3 : 4;
  if (!gram) ck(launch_rinv(rdt, c.R, m, m, c.X, h->stream));
  const int64_t W = wide_size(dtype);
  int worst = MN_OK;
  if (block) worst = solve_block(c, b, ldb, (int)nrhs, x, ldx, info);
  for (int64_t j = 0; j < (block ? 0 : nrhs); ++j) {
    const void* bj = (const char*)b + j * ldb * W;
    void* xj = (char*)x + j * ldx * W;
    const int s = solve_one(c, bj, xj, info);
    if (s > worst) worst = s;
  }
  ev_record(h, 8);
  if (info) {
    info->status = worst;
    if (h->events) {
      ck(hipEventSynchronize(h->ev[8]));
      float t = 0;
      (void)hipEventElapsedTime(&t, h->ev[0], h->ev[1]);
      info->stage_ms[0] = t;
      (void)hipEventElapsedTime(&t, h->ev[1], h->ev[2]);
      info->stage_ms[1] = t;
      (void)hipEventElapsedTime(&t, h->ev[3], h->ev[4]);
      info->stage_ms[2] = t;
      (void)hipEventElapsedTime(&t, h->ev[4], h->ev[5]);
      info->stage_ms[3] = t;
      (void)hipEventElapsedTime(&t, h->ev[0], h->ev[8]);
      info->stage_ms[7] = t;
    }
  }
  return worst;
}

// ----------------------------------------------------------------------------
// Batched systems, fused form: every stage of every system is one launch
// whose workgroups find their system through a prefix table (BGrid), and the
// systems iterate in lockstep with their own stop flags, so the host waits a
// few times per batch instead of several times per system.  Requires m <= 512
// for every system (fused A-pass) and the Gram route for R; systems whose idx
// is invalid or whose Gram factor is declined are solved afterwards one by one.
struct GridTable {
  std::vector<BGrid> g;
  int total = 0;
  size_t off = 0;  // offset (entries) in the uploaded table buffer
  void init(int n) { g.assign((size_t)n + 1, BGrid{0, 0, 1, 1}); }
  void finish() {
    int acc = 0;
    for (size_t i = 0; i + 1 < g.size(); ++i) {
      const int cnt = g[i].gx * g[i].gy * g[i].gz;
      g[i].start = acc;
      acc += cnt;
    }
    g.back() = BGrid{acc, 1, 1, 1};
    total = acc;
  }
};


// The fused form takes one bulk type for all systems: either no system has a
// single-precision copy or every system has one (a mix goes to the lanes).
bool fused_batch_ok(int dtype, int batch, const int64_t* m, const int64_t* N, const int64_t* l,
                    const void* const* A_lo, const mn_opts& o) {
  if (o.precond != 0 || o.batch_form == 1 || batch < 2 || o.hfactor) return false;
  for (int i = 0; i < batch; ++i)
    if (m[i] > kGramMaxRows) return false;
  // a length N = N1 2^k needs the fused form's kept-outputs-only sketch
  // (B = 16, 256 threads, l <= 2048)
  const int bulk = A_lo ? dtype + 1 : dtype;
  for (int i = 0; i < batch; ++i)
    if (!is_pow2(N[i]) && !(l[i] <= 2048 && sketch_pruned_groups(bulk, N[i], l[i], 16, 1) > 0)) return false;
  if (A_lo)
    for (int i = 0; i < batch; ++i)
      if (!A_lo[i]) return false;
  return true;
}

void fill_info_from_state(const PcgState& s, bool mixed, mn_info* info) {
  info->status = s.status;
  info->iters = s.iter_total;
  info->refine_steps = s.refine_steps;
  info->nrhs_done = s.status == MN_OK ? 1 : 0;
  const double rho = mixed ? s.outer_rho : s.rho;
  const double xi = mixed ? s.outer_xi : s.xi;
  info->cert_rel = xi > 0 ? std::sqrt(rho / xi) : 0.0;
  info->rho0 = s.rho0;
  info->rho = rho;
  info->xi = xi;
}

// Returns the per-system statuses in st_out; systems listed in redo still
// need a one-system solve.
void solve_batched_fused(mn_handle h, int dtype, int batch, const int64_t* m, const int64_t* n, const void* const* A,
                         const int64_t* lda, const void* const* A_lo, const void* const* b, const double* eps,
                         const int64_t* N, const int64_t* l, const void* const* d, const int32_t* const* idx,
                         const mn_opts& o, void* const* x, mn_info* info, std::vector<int>& st_out,
                         std::vector<int>& redo) {
  hipStream_t st = h->stream;
  // the passes' rows-per-lane classes run side by side
  const StreamFork* fork = handle_fork(h);
  const bool cplx = is_complex(dtype);
  const bool mixed = A_lo != nullptr || is_single(dtype);
  const int bulk = A_lo ? dtype + 1 : dtype;
  const int64_t W = wide_size(dtype);
  const int64_t be = dtype_size(bulk);
  const int64_t ces = is_single(bulk) ? 8 : 16;
  std::vector<BSys> hs((size_t)batch);
  // grids
  GridTable fill, map, sk_small, sk_cols, sk_rows, sk_ord, sk_pr[3], gram_s, rdiag, invd, gramR[4], gred, adjA, adjU,
      sum, fwdA, fwdU, cgs, cgp, vec, colm;
  for (GridTable* t : {&fill, &map, &sk_small, &sk_cols, &sk_rows, &sk_ord, &sk_pr[0], &sk_pr[1], &sk_pr[2], &gram_s,
                       &rdiag, &invd, &gramR[0], &gramR[1], &gramR[2], &gramR[3], &gred, &adjA, &adjU, &sum, &fwdA,
                       &fwdU, &cgs, &cgp, &vec, &colm})
    t->init(batch);
  int maxnbk = 0;
  size_t lds_small = 0, lds_cols = 0, lds_rows = 0, lds_pr = 0;
  // the fused passes read column-major copies of the bulk matrices (written
  // by the first pass) where all of them fit in half the free memory; the
  // copy also spares the padded re-layout of rows that are not 16-byte aligned
  bool use_cm = false;
  {
    double need = 0.0;
    for (int i = 0; i < batch; ++i) need += (double)(rup(m[i], 64) * n[i] * dtype_size(bulk));
    size_t fr = 0, tot = 0;
    use_cm = hipMemGetInfo(&fr, &tot) == hipSuccess && need <= 0.5 * (double)fr;
  }
  int64_t maxm = 0;
  std::vector<int64_t> wbytes((size_t)batch);
  for (int i = 0; i < batch; ++i) {
    BSys& q = hs[i];
    memset(&q, 0, sizeof(q));
    q.A = A[i];
    q.lda = lda[i];
    q.Ab = A_lo ? A_lo[i] : A[i];
    q.ldab = lda[i];
    q.m = m[i];
    q.n = n[i];
    q.N = N[i];
    q.l = l[i];
    q.b = b[i];
    q.x = x[i];
    q.d = d[i];
    q.idx = idx[i];
    q.ldx = rinv_ld(m[i]);
    maxm = std::max(maxm, m[i]);
    BGrid g0, g1, g2, g3;
    size_t a0, a1, a2, a3;
    b_plan_sketch(bulk, q, g0, g1, g2, g3, a0, a1, a2, a3);
    sk_small.g[i] = g0;
    sk_cols.g[i] = g1;
    sk_rows.g[i] = g2;
    const int kc = q.sk_kpt == 2 ? 0 : (q.sk_kpt == 4 ? 1 : (q.sk_kpt == 8 ? 2 : -1));
    for (int c = 0; c < 3; ++c) sk_pr[c].g[i] = c == kc ? g3 : BGrid{0, 0, 1, 1};
    sk_ord.g[i] = kc >= 0 ? BGrid{0, 1, 1, 1} : BGrid{0, 0, 1, 1};
    lds_small = std::max(lds_small, a0);
    lds_cols = std::max(lds_cols, a1);
    lds_rows = std::max(lds_rows, a2);
    lds_pr = std::max(lds_pr, a3);
    q.tw = twiddles(h, N[i], is_single(bulk));
    fill.g[i] = BGrid{0, (int)cdiv(N[i], 256), 1, 1};
    map.g[i] = BGrid{0, (int)cdiv(l[i], 256), 1, 1};
    gram_s.g[i] = BGrid{0, (int)cdiv(m[i], 128), 1, (int)cdiv(m[i], gram_col_block(bulk))};
    rdiag.g[i] = BGrid{0, 1, 1, 1};
    invd.g[i] = BGrid{0, (int)cdiv(m[i], 32), 1, 1};
    maxnbk = std::max(maxnbk, (int)cdiv(m[i], 32));
    BGrid gg, gr;
    // every bulk row start is 16-byte aligned (padded below if not)
    const int cls = b_plan_gram(bulk, q, gg, gr);
    b_plan_gram_res(dtype, q);
    for (int c = 0; c < 4; ++c) gramR[c].g[i] = c == cls ? gg : BGrid{0, 0, 1, 1};
    gred.g[i] = gr;
    BGrid ga, gs, gf;
    const bool al = b_aligned16(q.A, q.lda, dtype);
    b_plan_wide(dtype, al, q, ga, gs, gf);
    (al ? adjA : adjU).g[i] = ga;
    sum.g[i] = gs;
    (al ? fwdA : fwdU).g[i] = gf;
    cgs.g[i] = BGrid{0, (int)cdiv(m[i], 8), 1, 1};
    cgp.g[i] = BGrid{0, (int)cdiv(m[i], 16), 1, 1};
    vec.g[i] = BGrid{0, (int)cdiv(m[i], 256), 1, 1};
    const int64_t mm = m[i];
    // an unaligned bulk row start is re-laid with a padded leading dimension
    // (one extra pass over the bulk copy) so that the fused pass reads
    // 16-byte vectors
    const int64_t pad_ld = (use_cm || b_aligned16(q.Ab, q.ldab, bulk)) ? 0 : rup(n[i], std::max<int64_t>(16 / be, 1));
    if (use_cm) colm.g[i] = BGrid{0, (int)cdiv(n[i], b_colmajor_tw(bulk)), (int)(rup(mm, 64) / 64), 1};
    wbytes[i] = a256(pad_ld * mm * be) + (use_cm ? a256(rup(mm, 64) * n[i] * be) : 0) + a256(N[i] * 4) +
                a256(sketch_order_bytes(l[i], is_single(bulk))) + a256(l[i] * mm * be) +
                a256(b_sketch_work_elems(bulk, mm, N[i], l[i]) * ces) +
                2 * a256(mm * mm * W) + a256(q.ldx * q.ldx * W) + a256(chol_scratch_elems(mm) * W) +
                6 * a256(mm * W) + a256(kGramParts * mm * W) + a256(3 * mm * W) +
                a256((int64_t)q.gram_G * mm * W) + a256(n[i] * W) + a256((int64_t)q.adj_slabs * n[i] * W) +
                a256((int64_t)q.fwd_chunks * mm * W);
  }
  // chol[0]: the first diagonal tiles; chol[k + 1]: block step k
  std::vector<GridTable> chol((size_t)maxnbk), trtri((size_t)maxnbk);
  for (int k = 0; k < maxnbk; ++k) {
    chol[k].init(batch);
    trtri[k].init(batch);
    for (int i = 0; i < batch; ++i) {
      const int nb = (int)cdiv(m[i], 32);
      const int ks = k - 1;
      if (k == 0) chol[k].g[i] = BGrid{0, 1, 1, 1};
      else if (ks + 1 < nb) chol[k].g[i] = BGrid{0, (nb - ks - 1) + (nb - ks - 1) * (nb - ks) / 2, 1, 1};
      else chol[k].g[i] = BGrid{0, 0, 1, 1};
      // trtri[k]: block step k of the right-looking inverse
      if (k + 1 < nb) trtri[k].g[i] = BGrid{0, (k + 1) * (nb - k - 1), 1, 1};
      else trtri[k].g[i] = BGrid{0, 0, 1, 1};
    }
  }
  // mark the grids of systems outside a launch
  for (int i = 0; i < batch; ++i) {
    const bool al = b_aligned16(hs[i].A, hs[i].lda, dtype);
    if (al) {
      adjU.g[i].gx = 0;
      fwdU.g[i].gx = 0;
    } else {
      adjA.g[i].gx = 0;
      fwdA.g[i].gx = 0;
    }
  }
  std::vector<GridTable*> all = {&fill,     &map,      &sk_small, &sk_cols,  &sk_rows,  &sk_ord, &sk_pr[0],
                                 &sk_pr[1], &sk_pr[2], &gram_s,   &rdiag,    &invd,     &gramR[0], &gramR[1],
                                 &gramR[2], &gramR[3], &gred,     &adjA,     &adjU,     &sum,    &fwdA,
                                 &fwdU,     &cgs,      &cgp,      &vec,     &colm};
  for (auto& t : chol) all.push_back(&t);
  for (auto& t : trtri) all.push_back(&t);
  size_t nent = 0;
  for (GridTable* t : all) {
    t->finish();
    t->off = nent;
    nent += t->g.size();
  }
  // workspace: per-system slices, plus contiguous flags/diag/state arrays
  int64_t total = 0;
  std::vector<int64_t> base((size_t)batch);
  for (int i = 0; i < batch; ++i) {
    base[i] = total;
    total += wbytes[i];
  }
  char* wsb = (char*)ws(h, "batch_ws", (size_t)total);
  int32_t* flags = (int32_t*)ws(h, "batch_flags", (size_t)batch * 16);
  double* diag = (double*)ws(h, "batch_diag", (size_t)batch * 32);
  PcgState* states = (PcgState*)ws(h, "batch_states", (size_t)batch * sizeof(PcgState));
  for (int i = 0; i < batch; ++i) {
    BSys& q = hs[i];
    char* p = wsb + base[i];
    auto take = [&](int64_t bytes) {
      char* r = p;
      p += a256(bytes);
      return (void*)r;
    };
    const int64_t mm = m[i];
    if (use_cm) {
      q.ldt = rup(mm, 64);
      q.At = take(q.ldt * n[i] * be);
    } else if (!b_aligned16(q.Ab, q.ldab, bulk)) {
      const int64_t pld = rup(n[i], std::max<int64_t>(16 / be, 1));
      void* pad = take(pld * mm * be);
      ck(hipMemcpy2DAsync(pad, (size_t)(pld * be), q.Ab, (size_t)(q.ldab * be), (size_t)(n[i] * be), (size_t)mm,
                          hipMemcpyDeviceToDevice, st));
      q.Ab = pad;
      q.ldab = pld;
    }
    q.inv = (int32_t*)take(N[i] * 4);
    q.order = (int32_t*)take(sketch_order_bytes(l[i], is_single(bulk)));
    q.S = take(l[i] * mm * be);
    q.Y = take(b_sketch_work_elems(bulk, mm, N[i], l[i]) * ces);
    q.G = take(mm * mm * W);
    q.R = take(mm * mm * W);
    q.X = take(q.ldx * q.ldx * W);
    q.Yd = take(chol_scratch_elems(mm) * W);
    q.y = take(mm * W);
    q.r0 = take(mm * W);
    q.r1 = take(mm * W);
    q.p = take(mm * W);
    q.s = take(mm * W);
    q.y_outer = take(mm * W);
    q.q = take(kGramParts * mm * W);
    q.qpart = take((int64_t)q.gram_G * mm * W);
    q.w64 = take(n[i] * W);
    q.apart = take((int64_t)q.adj_slabs * n[i] * W);
    q.fpart = take((int64_t)q.fwd_chunks * mm * W);
    q.pw = take(3 * mm * W);
    q.flags = flags + 4 * i;
    q.diag = diag + 4 * i;
    q.st = states + i;
  }
  // upload descriptors and tables through pinned staging
  const size_t sys_bytes = sizeof(BSys) * (size_t)batch, tab_bytes = sizeof(BGrid) * nent;
  BSys* dsys = (BSys*)ws(h, "batch_sys", sys_bytes);
  BGrid* dtab = (BGrid*)ws(h, "batch_tab", tab_bytes);
  if (h->host_stage_bytes < sys_bytes + tab_bytes + (size_t)batch * sizeof(PcgState)) {
    ck(hipStreamSynchronize(st));
    if (h->host_stage) ck(hipHostFree(h->host_stage));
    h->host_stage = nullptr;
    h->host_stage_bytes = sys_bytes + tab_bytes + (size_t)batch * sizeof(PcgState) + 4096;
    ck(hipHostMalloc((void**)&h->host_stage, h->host_stage_bytes, hipHostMallocDefault));
  }
  char* hst = (char*)h->host_stage;
  memcpy(hst, hs.data(), sys_bytes);
  for (GridTable* t : all) memcpy(hst + sys_bytes + t->off * sizeof(BGrid), t->g.data(), t->g.size() * sizeof(BGrid));
  ck(hipMemcpyAsync(dsys, hst, sys_bytes, hipMemcpyHostToDevice, st));
  ck(hipMemcpyAsync(dtab, hst + sys_bytes, tab_bytes, hipMemcpyHostToDevice, st));
  ck(launch_fill0(flags, (int64_t)batch * 16, st));
  ck(hipStreamSynchronize(st));
  auto L = [&](GridTable& t) { return BLaunch{dsys, dtab + t.off, batch, t.total}; };
  const BLaunch none{dsys, dtab + fill.off, batch, 0};

  // idx check first: a system with an invalid idx takes no part in any later
  // launch (the sketch gathers through idx)
  ck(launch_b_prep(L(fill), L(map), st));
  ck(hipMemcpyAsync(hst, flags, (size_t)batch * 16, hipMemcpyDeviceToHost, st));
  ck(hipStreamSynchronize(st));
  std::vector<char> idx_bad((size_t)batch, 0);
  bool any_bad = false;
  for (int i = 0; i < batch; ++i) {
    idx_bad[i] = reinterpret_cast<const int32_t*>(hst)[4 * i] != 0;
    any_bad = any_bad || idx_bad[i];
  }
  if (any_bad) {
    for (GridTable* t : all) {
      if (t == &fill || t == &map) continue;
      for (int i = 0; i < batch; ++i)
        if (idx_bad[i]) t->g[i].gx = 0;
      t->finish();
      memcpy(hst + sys_bytes + t->off * sizeof(BGrid), t->g.data(), t->g.size() * sizeof(BGrid));
    }
    memcpy(hst, hs.data(), sys_bytes);
    ck(hipMemcpyAsync(dtab, hst + sys_bytes, tab_bytes, hipMemcpyHostToDevice, st));
    ck(hipStreamSynchronize(st));
  }
  // Steps 1-2: sketch, Gram matrix, Cholesky, diagonal range
  const BLaunch prl[3] = {L(sk_pr[0]), L(sk_pr[1]), L(sk_pr[2])};
  ck(launch_b_sketch(bulk, L(sk_small), L(sk_cols), L(sk_rows), L(sk_ord), prl, lds_small, lds_cols, lds_rows, lds_pr,
                     st));
  // the column-major copies on a side stream beside Step 2 (the first pass
  // then reads them instead of writing them); every way out of this call
  // leaves the stream behind them
  bool pre_cm = false;
  struct CmJoin {
    hipStream_t st;
    hipEvent_t e;
    const bool* on;
    ~CmJoin() {
      if (*on) (void)hipStreamWaitEvent(st, e, 0);
    }
  } cm_join{st, h->pre_ev[1], &pre_cm};
  if (use_cm && colm.total > 0) {
    ck(hipEventRecord(h->pre_ev[0], st));
    ck(hipStreamWaitEvent(fork->side[0], h->pre_ev[0], 0));
    ck(launch_b_colmajor(bulk, L(colm), fork->side[0]));
    ck(hipEventRecord(h->pre_ev[1], fork->side[0]));
    pre_cm = true;
  }
  ck(launch_b_gram_s(bulk, L(gram_s), st));
  for (int k = 0; k < maxnbk; ++k) ck(launch_b_chol_step(cplx, L(chol[k]), k - 1, st));
  ck(launch_b_rdiag(cplx, L(rdiag), st));
  // X = R^{-1}, then the condition estimate (gram_factor's rule)
  ck(launch_b_inv_diag(cplx, L(invd), st));
  for (int k = 0; k + 1 < maxnbk; ++k) ck(launch_b_trtri_step(cplx, L(trtri[k]), k, st));
  ck(launch_b_power(cplx, L(rdiag), 4, st));
  std::vector<int32_t> hflags((size_t)batch * 4);
  std::vector<double> hdiag((size_t)batch * 4);
  ck(hipMemcpyAsync(hst, flags, (size_t)batch * 16, hipMemcpyDeviceToHost, st));
  ck(hipMemcpyAsync(hst + (size_t)batch * 16, diag, (size_t)batch * 32, hipMemcpyDeviceToHost, st));
  ck(hipStreamSynchronize(st));
  memcpy(hflags.data(), hst, (size_t)batch * 16);
  memcpy(hdiag.data(), hst + (size_t)batch * 16, (size_t)batch * 32);
  std::vector<char> skip((size_t)batch, 0);
  std::vector<double> kap_of((size_t)batch, 0.0);
  st_out.assign((size_t)batch, MN_OK);
  for (int i = 0; i < batch; ++i) {
    const double mx = hdiag[4 * i], mn_ = hdiag[4 * i + 1], nf = hdiag[4 * i + 2];
    const bool bad_idx = idx_bad[i] != 0;
    const double pk = hdiag[4 * i + 3];
    double kap = mn_ > 0.0 ? mx / mn_ : 1e300;
    kap = (std::isfinite(pk) && pk > 0.0) ? std::max(kap, std::sqrt(pk)) : 1e300;
    const bool gram_ok = hflags[4 * i + 1] == 0 && nf == 0.0 && std::isfinite(mx) && mn_ > 0.0 &&
                         gram_accurate(l[i], is_single(bulk), kap);
    kap_of[i] = kap;
    if (bad_idx) {
      st_out[i] = -16;
      skip[i] = 1;
    } else if (!gram_ok) {
      redo.push_back(i);
      skip[i] = 1;
    }
  }
  // CG states (skipped systems start finished)
  std::vector<PcgState> hst_state((size_t)batch);
  for (int i = 0; i < batch; ++i) {
    PcgState& s0 = hst_state[i];
    memset(&s0, 0, sizeof(s0));
    s0.eps = mixed ? std::pow(10.0, -(double)(o.inner_digits ? o.inner_digits : 4))
                   : eps[i] * (skip[i] ? 1.0 : sigma_floor(l[i], kap_of[i]));
    s0.alpha = o.alpha;
    s0.l = (double)l[i];
    s0.N = (double)N[i];
    s0.eps_outer = eps[i];
    s0.rule = mixed ? 2 : o.stop_rule;
    s0.max_iter = o.max_iter;
    s0.max_refine = o.max_refine;
    if (skip[i]) {
      s0.done = 1;
      s0.outer_done = 1;
    }
  }
  auto read_states = [&]() {
    ck(hipMemcpyAsync(hst, states, (size_t)batch * sizeof(PcgState), hipMemcpyDeviceToHost, st));
    ck(hipStreamSynchronize(st));
    memcpy(hst_state.data(), hst, (size_t)batch * sizeof(PcgState));
  };
  memcpy(hst, hst_state.data(), (size_t)batch * sizeof(PcgState));
  ck(hipMemcpyAsync(states, hst, (size_t)batch * sizeof(PcgState), hipMemcpyHostToDevice, st));
  ck(hipStreamSynchronize(st));
  const size_t cg_lds = (size_t)maxm * W;
  int par = 0;
  if (pre_cm) ck(hipStreamWaitEvent(st, h->pre_ev[1], 0));
  bool at_written = pre_cm;
  auto all_done = [&](bool outer) {
    for (int i = 0; i < batch; ++i)
      if (!(outer ? hst_state[i].outer_done : hst_state[i].done)) return false;
    return true;
  };
  // One block of check_every lockstep iterations: per iteration the fused
  // pass of every system and its CG step.  Once the column-major copies are
  // written the block's launches are the same every time (the kernels read
  // each system's stop flag), so the block is captured once as a HIP graph
  // per parity of the r ping-pong and replayed (no memset or host transfer
  // inside the captured region); opts.graph = -1 launches every kernel.
  const int ce = o.check_every > 0 ? o.check_every : 8;
  auto enqueue_block = [&](hipStream_t s) {
    for (int it = 0; it < ce; ++it) {
      const BLaunch gl[4] = {L(gramR[0]), L(gramR[1]), L(gramR[2]), L(gramR[3])};
      // timing (mn_profile, launched blocks only): the fused passes of all
      // systems with their partial-sum reduction, as one interval
      const auto ev = s == st ? prof_pair(h, K_GRAM) : std::pair<hipEvent_t, hipEvent_t>{nullptr, nullptr};
      if (ev.first) ck(hipEventRecord(ev.first, s));
      ck(launch_b_gram(bulk, gl, L(gred), use_cm ? (at_written ? 2 : 1) : 0, s, fork));
      if (ev.second) ck(hipEventRecord(ev.second, s));
      at_written = true;
      ck(launch_b_cg(cplx, L(cgs), L(cgp), 0, 2, 0, par, cg_lds, s));
      par ^= 1;
    }
  };
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  struct GraphsOut {
    hipGraphExec_t* g;
    ~GraphsOut() {
      for (int k = 0; k < 2; ++k)
        if (g[k]) (void)hipGraphExecDestroy(g[k]);
    }
  } graphs_out{gexec};
  const bool use_graph = o.graph >= 0;
  auto replay_block = [&]() {
    const int p0 = par;
    if (!gexec[p0]) {
      // recorded on the handle's capture stream (the handle's own stream may
      // be the null stream, which cannot be captured); nothing runs there
      if (!h->cap_stream) ck(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
      hipStream_t cs = h->cap_stream;
      hipGraph_t g = nullptr;
      ck(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      try {
        enqueue_block(cs);
      } catch (HipFail) {
        (void)hipStreamEndCapture(cs, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      ck(hipStreamEndCapture(cs, &g));
      const hipError_t e = hipGraphInstantiate(&gexec[p0], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      ck(e);
      par = p0;  // the capture only recorded the block
    }
    ck(hipGraphLaunch(gexec[p0], st));
    par = p0 ^ (ce & 1);
  };
  auto inner_loop = [&]() {
    int guard = 0;
    while (true) {
      if (use_graph && (!use_cm || at_written)) replay_block();
      else enqueue_block(st);
      read_states();
      if (all_done(false)) break;
      if ((guard += ce) > o.max_iter + 2 * ce) break;  // the kernels cap iterations
    }
  };
  if (mixed) {
    ck(launch_b_zero_outer(cplx, L(vec), st));
    for (int outer = 0; outer <= o.max_refine + 1; ++outer) {
      // r = b - A (A* y_outer) in FP64: one fused pass over FP64 data (its
      // instances for single-precision problem data with m > 256 would spill
      // registers, so those keep the two passes A* then A); y_outer = 0 at
      // the first step, whose residual is b itself
      if (outer == 0) {
        ck(launch_b_cg(cplx, L(cgs), L(cgp), 1, 0, 1, par, cg_lds, st));
      } else if (!is_single(dtype)) {
        const BLaunch gl[4] = {L(gramR[0]), L(gramR[1]), L(gramR[2]), L(gramR[3])};
        ck(launch_b_gram_res(dtype, gl, L(gred), st, fork));
        ck(launch_b_cg(cplx, L(cgs), L(cgp), 1, 2, 1, par, cg_lds, st));
      } else {
        ck(launch_b_adj_wide(dtype, true, L(adjA), none, 0, 0, st));
        ck(launch_b_adj_wide(dtype, false, L(adjU), L(sum), 0, 0, st));
        ck(launch_b_fwd_wide(dtype, true, L(fwdA), st));
        ck(launch_b_fwd_wide(dtype, false, L(fwdU), st));
        ck(launch_b_cg(cplx, L(cgs), L(cgp), 1, 1, 1, par, cg_lds, st));
      }
      read_states();
      if (all_done(true)) break;
      inner_loop();
      ck(launch_b_refine(cplx, L(vec), st));
    }
    // x = A* y_outer
    ck(launch_b_adj_wide(dtype, true, L(adjA), none, 0, 1, st));
    ck(launch_b_adj_wide(dtype, false, L(adjU), L(sum), 0, 1, st));
  } else {
    ck(launch_b_cg(cplx, L(cgs), L(cgp), 1, 0, 0, par, cg_lds, st));
    inner_loop();
    ck(launch_b_adj_wide(dtype, true, L(adjA), none, 1, 1, st));
    ck(launch_b_adj_wide(dtype, false, L(adjU), L(sum), 1, 1, st));
  }
  read_states();
  for (int i = 0; i < batch; ++i) {
    if (skip[i]) continue;
    st_out[i] = hst_state[i].status;
    if (info) {
      memset(&info[i], 0, sizeof(mn_info));
      fill_info_from_state(hst_state[i], mixed, &info[i]);
      info[i].factor = 1;
      info[i].kappa_hat = kap_of[i];
    }
  }
}


int check_solve_args(mn_handle h, int dtype, int64_t m, int64_t n, const void* A, int64_t lda, const void* A_lo,
                     int64_t lda_lo, const void* b, int64_t ldb, int64_t nrhs, double eps, int64_t N, int64_t l,
                     const void* d, const int32_t* idx, const mn_opts& o, void* x, int64_t ldx) {
  if (!h) return -1;
  if (dtype < 0 || dtype > 3) return -2;
  if (m < 1 || m >= n || m > kMaxRows) return -3;
  if (n < 2) return -4;
  if (!A) return -5;
  if (lda < n) return -6;
  if (A_lo && is_single(dtype)) return -7;
  if (A_lo && lda_lo < n) return -8;
  if (!b) return -9;
  if (ldb < m) return -10;
  if (nrhs < 1 || nrhs > 64) return -11;
  if (!(eps > 0.0 && eps < 1.0)) return -12;
  if (!is_fft_len(N) || N < n || N > (1 << 22)) return -13;
  if (l <= m || l > N) return -14;
  // the sketch runs in the bulk precision (single with A_lo)
  if (!sketch_ok(A_lo ? dtype + 1 : dtype, N, l)) return -13;
  if (!d && idx) return -15;  // both NULL: the library draws
  if (d && !idx) return -16;
  if (!opts_valid(o)) return -17;
  if (!x) return -18;
  if (ldx < n) return -19;
  return 0;
}

}  // namespace

// =============================================================================
extern "C" {

int mn_create(mn_handle* hp, void* stream) {
  if (!hp) return -1;
  *hp = nullptr;
  mn_handle h = new mn_handle_s();
  try {
    h->stream = (hipStream_t)stream;
    ck(hipGetDevice(&h->device));
    // the allocation-free entry point's static array: its address on this
    // device, looked up once while the device is current
    ck(noalloc_init(h->device));
    ck(hipHostMalloc((void**)&h->host_state, sizeof(PcgState), hipHostMallocDefault));
    ck(hipHostMalloc((void**)&h->host_snap, 2 * sizeof(PcgState), hipHostMallocDefault));
    for (auto& e : h->snap_ev) ck(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ck(hipHostMalloc((void**)&h->host_blk, sizeof(BlkState), hipHostMallocDefault));
    ck(hipHostMalloc((void**)&h->host_flag, 64, hipHostMallocDefault));
    ck(hipHostMalloc((void**)&h->host_diag, 256, hipHostMallocDefault));
    for (auto& e : h->ev) ck(hipEventCreate(&e));
    for (auto& e : h->tev) ck(hipEventCreate(&e));
  } catch (HipFail f) {
    mn_destroy(h);
    return fail_hip(f.e);
  }
  *hp = h;
  return 0;
}

int mn_destroy(mn_handle h) {
  if (!h) return -1;
  for (mn_handle c : h->lanes) mn_destroy(c);
  h->lanes.clear();
  (void)hipStreamSynchronize(h->stream);
  for (auto& kv : h->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  for (auto& kv : h->tw)
    if (kv.second.p) (void)hipFree(kv.second.p);
  if (h->host_state) (void)hipHostFree(h->host_state);
  if (h->host_snap) (void)hipHostFree(h->host_snap);
  for (auto& e : h->snap_ev)
    if (e) (void)hipEventDestroy(e);
  if (h->host_blk) (void)hipHostFree(h->host_blk);
  if (h->host_stage) (void)hipHostFree(h->host_stage);
  if (h->host_draw) (void)hipHostFree(h->host_draw);
  if (h->host_flag) (void)hipHostFree(h->host_flag);
  if (h->host_diag) (void)hipHostFree(h->host_diag);
  for (auto& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : h->tev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : h->pool) (void)hipEventDestroy(e);
  if (h->owns_stream && h->stream) (void)hipStreamDestroy(h->stream);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (auto& sd : h->fork.side)
    if (sd) (void)hipStreamDestroy(sd);
  for (auto& e : h->fork.ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : h->pre_ev)
    if (e) (void)hipEventDestroy(e);
  delete h;
  return 0;
}

int mn_set_stream(mn_handle h, void* stream) {
  if (!h) return -1;
  h->stream = (hipStream_t)stream;
  return 0;
}

const char* mn_status_string(int status) {
  switch (status) {
    case MN_OK: return "success";
    case MN_RANK_DEFICIENT: return "sketch numerically rank-deficient (redraw d, idx; A may not have full rank)";
    case MN_NOT_CONVERGED: return "iteration cap reached before the stopping rule was met";
    case MN_HIP_ERROR: return "HIP runtime error";
    case MN_NONFINITE: return "non-finite value in the input or an intermediate";
  }
  if (status < 0) return "invalid argument (-status is its 1-based position)";
  return "unknown status";
}

const char* mn_last_hip_error(void) { return g_last_hip_error.c_str(); }

int mn_profile(mn_handle h, int enable) {
  if (!h) return -1;
  try {
    ck(hipStreamSynchronize(h->stream));
  } catch (HipFail f) {
    return fail_hip(f.e);
  }
  h->prof = enable > 0;
  h->prof_every = enable > 0 ? enable : 1;
  h->pool_used = 0;
  h->recs.clear();
  std::fill(h->prof_seen, h->prof_seen + 8, 0);
  return 0;
}

int mn_profile_read(mn_handle h, const char* kernel, int64_t* count, double* total_ms) {
  if (!h) return -1;
  if (!kernel) return -2;
  if (!count) return -3;
  if (!total_ms) return -4;
  int kid = -1;
  for (int i = 0; i < (int)(sizeof(kKernelNames) / sizeof(kKernelNames[0])); ++i)
    if (strcmp(kernel, kKernelNames[i]) == 0) kid = i;
  if (kid < 0) return -2;
  *count = 0;
  *total_ms = 0.0;
  try {
    ck(hipStreamSynchronize(h->stream));
    for (auto& r : h->recs) {
      if (r.kid != kid) continue;
      float t = 0.f;
      ck(hipEventElapsedTime(&t, h->pool[r.ev], h->pool[r.ev + 1]));
      *count += 1;
      *total_ms += t;
    }
  } catch (HipFail f) {
    return fail_hip(f.e);
  }
  return 0;
}

int mn_plans_save(mn_handle h, const char* path) {
  if (!h) return -1;
  if (!path) return -2;
  FILE* f = fopen(path, "w");
  if (!f) return -2;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  fprintf(f, "{\n  \"format\": \"minnorm-plans-1\",\n  \"plans\": {");
  bool first = true;
  for (auto& kv : h->plans) {
    fprintf(f, "%s\n    \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
    first = false;
  }
  fprintf(f, "\n  },\n  \"best_ms\": {");
  first = true;
  for (auto& kv : h->plan_ms) {
    fprintf(f, "%s\n    \"%s\": %.6g", first ? "" : ",", kv.first.c_str(), (double)kv.second);
    first = false;
  }
  fprintf(f, "\n  }\n}\n");
  const bool ok = fclose(f) == 0;
  return ok ? 0 : -2;
}

int mn_plans_load(mn_handle h, const char* path) {
  if (!h) return -1;
  if (!path) return -2;
  FILE* f = fopen(path, "r");
  if (!f) return -2;
  std::string txt;
  char buf[4096];
  size_t k;
  while ((k = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, k);
  fclose(f);
  // the "plans" object: "key": integer pairs
  const size_t at = txt.find("\"plans\"");
  if (at == std::string::npos) return -2;
  size_t i = txt.find('{', at);
  const size_t end = i == std::string::npos ? std::string::npos : txt.find('}', i);
  if (end == std::string::npos) return -2;
  std::map<std::string, int> got;
  while (true) {
    const size_t q0 = txt.find('"', i);
    if (q0 == std::string::npos || q0 > end) break;
    const size_t q1 = txt.find('"', q0 + 1);
    if (q1 == std::string::npos || q1 > end) return -2;
    const size_t colon = txt.find(':', q1);
    if (colon == std::string::npos || colon > end) return -2;
    char* stop = nullptr;
    const long v = strtol(txt.c_str() + colon + 1, &stop, 10);
    if (stop == txt.c_str() + colon + 1) return -2;
    got[txt.substr(q0 + 1, q1 - q0 - 1)] = (int)v;
    i = (size_t)(stop - txt.c_str());
  }
  std::lock_guard<std::mutex> lk(g_plan_mu);
  for (auto& kv : got) h->plans[kv.first] = kv.second;
  return (int)got.size() >= 0 ? 0 : -2;
}

int mn_plans_count(mn_handle h) {
  if (!h) return -1;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  return (int)h->plans.size();
}

int64_t mn_workspace_bytes(mn_handle h) {
  if (!h) return -1;
  int64_t t = 0;
  for (auto& kv : h->bufs) t += (int64_t)kv.second.bytes;
  for (auto& kv : h->tw) t += kv.second.N * (kv.first.second ? 8 : 16);
  return t;
}

int srft_sketch(mn_handle h, int dtype, int64_t m, int64_t n, const void* A, int64_t lda, int64_t N, int64_t l,
                const void* d, const int32_t* idx, void* S, int64_t lds) {
  if (!h) return -1;
  if (dtype < 0 || dtype > 3) return -2;
  if (m < 1) return -3;
  if (n < 1) return -4;
  if (!A) return -5;
  if (lda < n) return -6;
  if (!is_fft_len(N) || N < n || N > (1 << 22)) return -7;
  if (l < 1 || l > N) return -8;
  if (!sketch_ok(dtype, N, l)) return -7;
  if (!d) return -9;
  if (!idx) return -10;
  if (!S) return -11;
  if (lds < l) return -12;
  try {
    int32_t* inv = nullptr;
    if (!prepare_idx(h, idx, l, N, &inv)) return -10;
    run_sketch(h, dtype, m, n, A, lda, N, l, d, idx, inv, S, lds);
    ck(hipGetLastError());
  } catch (HipFail f) {
    return fail_hip(f.e);
  }
  return 0;
}

int minnorm_steps23(mn_handle h, int dtype, int64_t m, int64_t n, const void* A, int64_t lda, const void* b,
                    int64_t N, int64_t l, const void* d, const int32_t* idx, void* z, void* c, double* checks) {
  if (!h) return -1;
  if (dtype < 0 || dtype > 3) return -2;
  if (m < 1 || m >= n || m > kMaxRows) return -3;
  if (n < 2) return -4;
  if (!A) return -5;
  if (lda < n) return -6;
  if (!b) return -7;
  if (!is_pow2(N) || N < n || N > (1 << 22)) return -8;
  if (l <= m || l > N) return -9;
  if (!d) return -10;
  if (!idx) return -11;
  if (!z) return -12;
  if (!c) return -13;
  hipStream_t st = h->stream;
  const bool cplx = is_complex(dtype);
  const int wdt = cplx ? MN_C128 : MN_F64;
  const int64_t W = wide_size(dtype);
  try {
    // Steps 1-2 as the solve takes them: sketch, then R (Gram route when
    // accepted, else Householder) and X = R^{-1} in FP64
    int32_t* inv = nullptr;
    if (!prepare_idx(h, idx, l, N, &inv)) return -11;
    void* S = ws(h, "S", (size_t)(l * m * dtype_size(dtype)));
    run_sketch(h, dtype, m, n, A, lda, N, l, d, idx, inv, S, l);
    const int64_t ldxi = rinv_ld(m);
    void* X = ws(h, "Xinv", (size_t)(ldxi * ldxi * W));
    void* R64 = ws(h, "R64", (size_t)(m * m * W));
    if (!gram_factor(h, dtype, l, m, S, l, R64, nullptr, X, ldxi)) {
      void* R = ws(h, "R", (size_t)(m * m * dtype_size(dtype)));
      const int rs = run_qr(h, dtype, l, m, S, l, R, m);
      if (rs != MN_OK) return rs;
      ck(launch_rinv(dtype, R, m, m, X, st));
    }
    // Step 2: z = S X X* b;  Step 3: c = T* z
    void* g = ws(h, "st_g", (size_t)(m * W));
    void* u = ws(h, "st_u", (size_t)(m * W));
    ck(launch_st_solve(cplx, X, ldxi, m, b, g, u, st));
    void* y = ws(h, "st_y", (size_t)(N * W));
    ck(launch_fill0(y, N * W, st));
    ck(launch_st_z(dtype, S, l, l, m, u, idx, z, y, st));
    void* ones = ws(h, "st_ones", (size_t)(N * W));
    int32_t* iota = (int32_t*)ws(h, "st_iota", (size_t)(N * 4));
    ck(launch_st_ones_iota(cplx, N, ones, iota, st));
    int32_t* inv_all = nullptr;
    if (!prepare_idx(h, iota, N, N, &inv_all)) return MN_HIP_ERROR;
    void* t = ws(h, "st_t", (size_t)(N * W));
    run_sketch(h, wdt, 1, N, y, N, N, N, ones, iota, inv_all, t, N);
    ck(launch_st_c(cplx, t, d, N, c, st));
    if (checks) {
      // ||A c - b|| / ||b|| (FP64 products of A's stored values), ||z||, ||c||
      FwdArgs fa{};
      fa.A = A;
      fa.lda = lda;
      fa.m = m;
      fa.n = n;
      fa.w = c;
      fa.qpart = ws(h, "qpart", (size_t)((kMaxChunks > kGramMaxWg ? kMaxChunks : kGramMaxWg) * m * W));
      int chunks = 1;
      fa.chunks_out = &chunks;
      ck(launch_gemv_fwd(dtype, true, fa, st));
      double* out = (double*)ws(h, "st_out", 64);
      ck(launch_st_resid(cplx, fa.qpart, chunks, m, b, out, st));
      double* nz = out + 2;
      ck(launch_st_resid(cplx, nullptr, 0, l, z, nz, st));   // ||z||^2 (as ||z - 0||^2)
      ck(launch_st_resid(cplx, nullptr, 0, N, c, nz + 2, st));
      ck(hipMemcpyAsync(h->host_diag, out, 6 * sizeof(double), hipMemcpyDeviceToHost, st));
      ck(hipStreamSynchronize(st));
      checks[0] = h->host_diag[1] > 0 ? std::sqrt(h->host_diag[0] / h->host_diag[1]) : std::sqrt(h->host_diag[0]);
      checks[1] = std::sqrt(h->host_diag[3]);
      checks[2] = std::sqrt(h->host_diag[5]);
    } else {
      ck(hipStreamSynchronize(st));
    }
  } catch (HipFail f) {
    return fail_hip(f.e);
  }
  return 0;
}

int srft_sketch_h(mn_handle h, int dtype, int64_t m, int64_t n, const void* A, int64_t lda, int64_t N, int64_t l,
                  const void* d, const int32_t* idx, const mn_hfactor* H, void* S, int64_t lds) {
  if (!h) return -1;
  if (dtype < 0 || dtype > 3) return -2;
  if (m < 1) return -3;
  if (n < 1) return -4;
  if (!A) return -5;
  if (lda < n) return -6;
  if (!is_fft_len(N) || N < n || N > (1 << 22)) return -7;
  if (l < 1 || l > N) return -8;
  if (!sketch_ok(dtype, N, l)) return -7;
  if (!d) return -9;
  if (!idx) return -10;
  if (!H || !H->theta || !H->perm || !H->zeta || !H->theta_t || !H->perm_t || !H->zeta_t) return -11;
  if (!S) return -12;
  if (lds < l) return -13;
  try {
    if (!hfactor_valid(h, H, N)) return -11;
    int32_t* inv = nullptr;
    if (!prepare_idx(h, idx, l, N, &inv)) return -10;
    run_sketch(h, dtype, m, n, A, lda, N, l, d, idx, inv, S, lds, nullptr, nullptr, H);
    ck(hipGetLastError());
  } catch (HipFail f) {
    return fail_hip(f.e);
  }
  return 0;
}

int srft_sketch_noalloc(mn_handle h, int dtype, int64_t m, int64_t n, const void* A, int64_t lda, int64_t N,
                        int64_t l, const void* d, const int32_t* idx, void* S, int64_t lds) {
  if (!h) return -1;
  if (dtype < 0 || dtype > 3) return -2;
  if (m < 1) return -3;
  if (n < 1) return -4;
  if (!A) return -5;
  if (lda < n) return -6;
  if (!is_pow2(N) || N < n || N > kNoAllocMaxN) return -7;
  if (l < 1 || l > N) return -8;
  if (!d) return -9;
  if (!idx) return -10;
  if (!S) return -11;
  if (lds < l) return -12;
  unsigned char* base = (unsigned char*)noalloc_ptr(h->device);
  if (!base) {
    g_last_hip_error = "the allocation-free workspace was not set up on this device";
    return MN_HIP_ERROR;
  }
  const bool single = is_single(dtype);
  // layout of the static array: twiddles | inverse map | flag | order and
  // kept-output table (sketch_order_bytes(l)) | work
  unsigned char* tw = base;
  int32_t* inv = (int32_t*)(base + kNoAllocTwBytes);
  int32_t* bad = (int32_t*)(base + kNoAllocTwBytes + kNoAllocIdxBytes);
  int32_t* order = (int32_t*)(base + kNoAllocTwBytes + kNoAllocIdxBytes + 256);
  const int64_t order_bytes = rup(sketch_order_bytes(l, is_single(dtype)), 256);
  unsigned char* work = (unsigned char*)order + order_bytes;
  const int64_t work_bytes = kNoAllocBytes - (work - base);
  if (twiddle_entries(N) * (single ? 8 : 16) > kNoAllocTwBytes) return -7;
  try {
    if (noalloc_twiddle_swap(h->device, (N << 1) | (single ? 1 : 0))) {
      const hipError_t e = launch_twiddles(single, N, tw, h->stream);
      if (e != hipSuccess) {
        noalloc_twiddle_swap(h->device, -1);
        throw HipFail{e};
      }
    }
    int32_t* inv_out = nullptr;
    if (!prepare_idx(h, idx, l, N, &inv_out, inv, bad)) return -10;
    const SketchArena ar{tw, order, work, work_bytes};
    run_sketch(h, dtype, m, n, A, lda, N, l, d, idx, inv_out, S, lds, nullptr, &ar);
    ck(hipGetLastError());
  } catch (HipFail f) {
    return fail_hip(f.e);
  }
  return 0;
}

int srft_draw(mn_handle h, int dtype, uint64_t seed, int32_t draw, int32_t sys, int64_t N, int64_t l, void* d,
              int32_t* idx) {
  if (!h) return -1;
  if (dtype < 0 || dtype > 3) return -2;
  if (draw < 0) return -4;
  if (sys < 0) return -5;
  if (N < 1 || N > (1 << 22)) return -6;
  if (l < 1 || l > N) return -7;
  if (!d) return -8;
  if (!idx) return -9;
  try {
    draw_srft_into(h, is_complex(dtype), seed, draw, sys, N, l, d, idx);
  } catch (HipFail f) {
    return fail_hip(f.e);
  }
  return 0;
}

int build_preconditioner(mn_handle h, int dtype, int64_t l, int64_t m, const void* S, int64_t lds, void* R,
                         int64_t ldr) {
  if (!h) return -1;
  if (dtype < 0 || dtype > 3) return -2;
  if (m < 1) return -4;
  if (l < m) return -3;
  if (!S) return -5;
  if (lds < l) return -6;
  if (!R) return -7;
  if (ldr < m) return -8;
  try {
    return run_qr(h, dtype, l, m, S, lds, R, ldr);
  } catch (HipFail f) {
    return fail_hip(f.e);
  }
}

int minnorm_solve(mn_handle h, int dtype, int64_t m, int64_t n, const void* A, int64_t lda, const void* A_lo,
                  int64_t lda_lo, const void* b, int64_t ldb, int64_t nrhs, double eps, int64_t N, int64_t l,
                  const void* d, const int32_t* idx, const mn_opts* opts, void* x, int64_t ldx, mn_info* info) {
  const mn_opts o = resolve_opts(opts);
  const int bad = check_solve_args(h, dtype, m, n, A, lda, A_lo, lda_lo, b, ldb, nrhs, eps, N, l, d, idx, o, x, ldx);
  if (bad) return bad;
  try {
    return solve_impl(h, dtype, m, n, A, lda, A_lo, lda_lo, b, ldb, nrhs, eps, N, l, d, idx, o, x, ldx, info);
  } catch (HipFail f) {
    if (info) info->status = MN_HIP_ERROR;
    return fail_hip(f.e);
  }
}

int minnorm_solve_batched(mn_handle h, int dtype, int32_t batch, const int64_t* m, const int64_t* n,
                          const void* const* A, const int64_t* lda, const void* const* A_lo, const void* const* b,
                          const double* eps, const int64_t* N, const int64_t* l, const void* const* d,
                          const int32_t* const* idx, const mn_opts* opts, void* const* x, mn_info* info) {
  if (!h) return -1;
  if (dtype < 0 || dtype > 3) return -2;
  if (batch < 1) return -3;
  if (!m) return -4;
  if (!n) return -5;
  if (!A) return -6;
  if (!lda) return -7;
  if (!b) return -9;
  if (!eps) return -10;
  if (!N) return -11;
  if (!l) return -12;
  if (!d && idx) return -13;  // both NULL: the library draws every system's
  if (d && !idx) return -14;
  if (!x) return -16;
  const mn_opts o = resolve_opts(opts);
  if (!opts_valid(o)) return -15;
  // argument checks for every system before any work is enqueued
  // minnorm_solve argument positions -> positions in this call
  static const int remap[20] = {0, -1, -2, -4, -5, -6, -7, -8, -7, -9, -4, -3, -10, -11, -12, -13, -14, -15, -16, -5};
  for (int32_t i = 0; i < batch; ++i) {
    const void* alo = A_lo ? A_lo[i] : nullptr;
    const int e = check_solve_args(h, dtype, m[i], n[i], A[i], lda[i], alo, lda[i], b[i], m[i], 1, eps[i], N[i],
                                   l[i], d ? d[i] : nullptr, idx ? idx[i] : nullptr, o, x[i], n[i]);
    if (e) return remap[-e];
  }
  // the library's own draws: every system's (d, idx) with draw 0 and sys = i
  // for the fused form (redraws happen in the one-system solves of the
  // systems it leaves); the lanes draw inside their one-system solves
  std::vector<const void*> dv;
  std::vector<const int32_t*> iv;
  const bool lib_draw = d == nullptr;
  auto d_of = [&](int i) -> const void* { return lib_draw ? nullptr : d[i]; };
  auto idx_of = [&](int i) -> const int32_t* { return lib_draw ? nullptr : idx[i]; };
  if (fused_batch_ok(dtype, batch, m, N, l, A_lo, o)) {
    std::vector<int> stv, redo;
    try {
      if (lib_draw) {
        int64_t dn = 0, in = 0;
        for (int32_t i = 0; i < batch; ++i) {
          dn += a256(N[i] * (is_complex(dtype) ? 16 : 8));
          in += a256(l[i] * 4);
        }
        char* dbase = (char*)ws(h, "bdraw_d", (size_t)dn);
        char* ibase = (char*)ws(h, "bdraw_idx", (size_t)in);
        int64_t* tab_dev = (int64_t*)ws(h, "bdraw_tab", (size_t)(2 * (int64_t)batch * 8));
        void* const d0 = dbase;
        int32_t* const i0 = (int32_t*)ibase;
        dv.resize(batch);
        iv.resize(batch);
        for (int32_t i = 0; i < batch; ++i) {
          dv[i] = dbase;
          iv[i] = (const int32_t*)ibase;
          dbase += a256(N[i] * (is_complex(dtype) ? 16 : 8));
          ibase += a256(l[i] * 4);
        }
        draw_srft_batch(h, is_complex(dtype), o.seed, batch, N, l, d0, i0, tab_dev);
      }
      solve_batched_fused(h, dtype, batch, m, n, A, lda, A_lo, b, eps, N, l, lib_draw ? dv.data() : d,
                          lib_draw ? iv.data() : idx, o, x, info, stv, redo);
      for (int i : redo) {
        const void* alo = A_lo ? A_lo[i] : nullptr;
        stv[i] = solve_impl(h, dtype, m[i], n[i], A[i], lda[i], alo, lda[i], b[i], m[i], 1, eps[i], N[i], l[i],
                            d_of(i), idx_of(i), o, x[i], n[i], info ? &info[i] : nullptr, i);
      }
    } catch (HipFail f) {
      return fail_hip(f.e);
    }
    int worst = MN_OK, argerr = 0;
    for (int32_t i = 0; i < batch; ++i) {
      if (stv[i] == -16) {
        argerr = -14;
        if (info) {
          memset(&info[i], 0, sizeof(mn_info));
          info[i].status = -14;
        }
      } else if (stv[i] > worst) {
        worst = stv[i];
      }
    }
    return argerr ? argerr : worst;
  }
  // Systems run concurrently on `streams` lanes (child handles, each with its
  // own stream, workspace and host thread), longest first; each lane solves
  // its systems one after another.  Lanes start after the work already
  // enqueued on the handle's stream.
  const int nl = std::min<int>(batch, o.streams);
  try {
    while ((int)h->lanes.size() < nl) {
      hipStream_t s = nullptr;
      ck(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      mn_handle c = nullptr;
      const int e = mn_create(&c, s);
      if (e) {
        (void)hipStreamDestroy(s);
        return e;
      }
      c->owns_stream = true;
      c->parent = h;
      h->lanes.push_back(c);
    }
    ck(hipEventRecord(h->ev[6], h->stream));
    for (int k = 0; k < nl; ++k) ck(hipStreamWaitEvent(h->lanes[k]->stream, h->ev[6], 0));
  } catch (HipFail f) {
    return fail_hip(f.e);
  }
  std::vector<int> order(batch);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return m[a] * n[a] > m[b] * n[b]; });
  std::vector<int> st(batch, MN_OK);
  std::atomic<int> next{0};
  auto work = [&](int k) {
    mn_handle c = h->lanes[k];
    if (hipSetDevice(h->device) != hipSuccess) return;
    while (true) {
      const int j = next.fetch_add(1);
      if (j >= batch) break;
      const int i = order[j];
      const void* alo = A_lo ? A_lo[i] : nullptr;
      int s;
      try {
        s = solve_impl(c, dtype, m[i], n[i], A[i], lda[i], alo, lda[i], b[i], m[i], 1, eps[i], N[i], l[i], d_of(i),
                       idx_of(i), o, x[i], n[i], info ? &info[i] : nullptr, i);
      } catch (HipFail f) {
        s = fail_hip(f.e);
      }
      if (info) info[i].status = s == -16 ? -14 : s;
      st[i] = s;
    }
  };
  std::vector<std::thread> th;
  for (int k = 1; k < nl; ++k) th.emplace_back(work, k);
  work(0);
  for (auto& t : th) t.join();
  int worst = MN_OK;
  int argerr = 0;
  for (int32_t i = 0; i < batch; ++i) {
    if (st[i] == -16) argerr = -14;  // idx of this system failed the device-side check
    else if (st[i] > worst) worst = st[i];
  }
  try {
    for (int k = 0; k < nl; ++k) {
      ck(hipEventRecord(h->lanes[k]->ev[7], h->lanes[k]->stream));
      ck(hipStreamWaitEvent(h->stream, h->lanes[k]->ev[7], 0));
    }
  } catch (HipFail f) {
    return fail_hip(f.e);
  }
  return argerr ? argerr : worst;
}

}  // extern "C"
